"""Dominance reductions on the GPU (kz_dominance, through the C ABI) against
the oracle (section 4.3, Definitions 4.3.1 and 4.3.2, Algorithms 1 and 2 as
read in oracle/kz_oracle_ext.c): masks, surviving adjacency and counts are
equal, on random graphs of every density, word-boundary sizes, the
thesis's evaluation sizes and the degenerate cases; bad inputs get the
status the header documents."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import dom_edge, dom_vertex  # noqa: E402
from paper_2212_00574_amd import inputs  # noqa: E402
from paper_2212_00574_amd.binding import (KZ_DOM_EDGE, KZ_DOM_VERTEX, Kernelizer, kz_dom_workspace_bytes,  # noqa: E402
                                          kz_dominance)

DEV = torch.device("cuda", 0)
KZ_EINVAL, KZ_EASYM, KZ_ESELFLOOP, KZ_ETOOLARGE = -1, -4, -5, -10


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def kz():
    k = Kernelizer(0)
    yield k
    k.close()


def random_graph(rng, n, p):
    a = (rng.random((n, n)) < p).astype(np.uint8)
    a = np.triu(a, 1)
    return a + a.T


def run(kz, adj, mode):
    n = adj.shape[0]
    rows = torch.from_numpy(inputs.dense_to_rows(adj).view(np.int64)).to(DEV)
    vm, em, res = kz.dominance(rows, mode)
    torch.cuda.synchronize()
    out = inputs.rows_to_dense(em.cpu().numpy(), n) if n else np.zeros((0, 0), np.uint8)
    return vm.cpu().numpy(), out, res


def check(kz, adj, ctx):
    n = adj.shape[0]
    ov_adj, ov_alive, ov = dom_vertex(adj)
    vm, out, res = run(kz, adj, KZ_DOM_VERTEX)
    assert res["status"] == 0, ctx
    assert np.array_equal(vm, ov_alive), ctx
    assert np.array_equal(out, ov_adj), ctx
    assert res["deleted_vertices"] == ov["deleted_vertices"] and res["deleted_edges"] == ov["deleted_edges"], ctx
    assert res["sweeps"] == ov["sweeps"] and res["events"] == ov["steps"], ctx
    assert res["input_edges"] == int(adj.sum()) // 2, ctx
    oe_adj, oe = dom_edge(adj)
    vm, out, res = run(kz, adj, KZ_DOM_EDGE)
    assert res["status"] == 0, ctx
    assert vm.all(), ctx
    assert np.array_equal(out, oe_adj), ctx
    assert res["deleted_edges"] == oe["deleted_edges"] and res["sweeps"] == oe["sweeps"], ctx


@pytest.mark.parametrize("seed", range(4))
def test_random_graphs_match_oracle(kz, seed):
    rng = np.random.default_rng(50 + seed)
    say("dominance: random graphs, seed", seed)
    for i in range(40):
        n = int(rng.integers(1, 200))
        check(kz, random_graph(rng, n, float(rng.uniform(0.02, 0.98))), (seed, i, n))


def test_word_boundaries(kz):
    rng = np.random.default_rng(9)
    for n in (63, 64, 65, 127, 128, 129, 191, 192, 193):
        for p in (0.1, 0.5, 0.95):
            check(kz, random_graph(rng, n, p), (n, p))


@pytest.mark.parametrize("n", [100, 300, 500])
def test_thesis_evaluation_sizes(kz, n):
    say("dominance: evaluation graph n =", n)
    check(kz, inputs.dominance_graph(n, 0), n)


def test_degenerate_graphs(kz):
    for n in (1, 2, 5, 70):
        check(kz, np.zeros((n, n), np.uint8), ("empty", n))
        full = np.ones((n, n), np.uint8) - np.eye(n, dtype=np.uint8)
        check(kz, full, ("complete", n))
    vm, em, res = kz.dominance(torch.empty((0, 1), dtype=torch.int64, device=DEV), KZ_DOM_VERTEX)
    assert res["status"] == 0 and res["deleted_vertices"] == 0


def test_in_place_and_statuses(kz):
    rng = np.random.default_rng(4)
    adj = random_graph(rng, 90, 0.4)
    n, R = 90, 2
    ws = torch.empty(kz_dom_workspace_bytes(n), dtype=torch.uint8, device=DEV)
    vm = torch.empty(n, dtype=torch.uint8, device=DEV)
    rows = torch.from_numpy(inputs.dense_to_rows(adj).view(np.int64)).to(DEV)
    res = kz_dominance(kz.ctx, KZ_DOM_EDGE, n, rows.data_ptr(), R, ws.data_ptr(), ws.numel(), vm.data_ptr(),
                       rows.data_ptr(), None)
    torch.cuda.synchronize()
    ref, _ = dom_edge(adj)
    assert res.status == 0 and np.array_equal(inputs.rows_to_dense(rows.cpu().numpy(), n), ref)

    def status(a, rw=None, mode=KZ_DOM_VERTEX, wsb=None):
        rws = inputs.dense_to_rows(a).view(np.int64)
        if rw is not None and rw > rws.shape[1]:
            rws = np.concatenate([rws, np.zeros((rws.shape[0], rw - rws.shape[1]), np.int64)], axis=1)
        t = torch.from_numpy(np.ascontiguousarray(rws)).to(DEV)
        em = torch.empty_like(t)
        v = torch.empty(a.shape[0], dtype=torch.uint8, device=DEV)
        r = kz_dominance(kz.ctx, mode, a.shape[0], t.data_ptr(), t.shape[1] if rw is None else rw, ws.data_ptr(),
                         ws.numel() if wsb is None else wsb, v.data_ptr(), em.data_ptr(), None)
        torch.cuda.synchronize()
        return r.status

    g = random_graph(rng, 70, 0.3)
    assert status(g) == 0
    bad = g.copy()
    bad[3, 50] = 1 - bad[3, 50]
    assert status(bad) == KZ_EASYM and status(bad, mode=KZ_DOM_EDGE) == KZ_EASYM
    loop = g.copy()
    loop[7, 7] = 1
    assert status(loop) == KZ_ESELFLOOP
    # a bit in a padding column (beyond n) of a row
    rws = inputs.dense_to_rows(g).view(np.int64).copy()
    rws[5, 1] |= np.int64(1) << np.int64(20)
    t = torch.from_numpy(rws).to(DEV)
    em = torch.empty_like(t)
    v = torch.empty(70, dtype=torch.uint8, device=DEV)
    r = kz_dominance(kz.ctx, KZ_DOM_VERTEX, 70, t.data_ptr(), 2, ws.data_ptr(), ws.numel(), v.data_ptr(),
                     em.data_ptr(), None)
    assert r.status == KZ_EINVAL
    assert status(g, rw=1) == KZ_EINVAL          # fewer words than ceil(n / 64)
    assert status(g, rw=1100) == KZ_ETOOLARGE    # rows beyond 1024 words
    assert status(g, wsb=16) == -6              # KZ_EWORKSPACE
    assert status(g, mode=7) == KZ_EINVAL


def test_evaluation_set_full_size(kz):
    """The thesis's ten evaluation sizes (n = 100..1900), both modes, against
    the oracle's fixture (tests/golden/dom_seed0.json, written by
    tests/golden/make_golden.py dom): SHA-256 of vmask || surviving bit rows ||
    [sweeps, deleted vertices, deleted edges, events]."""
    import hashlib
    import json
    import os
    fx = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "dom_seed0.json")))
    for rec in fx["graphs"]:
        n = rec["n"]
        say("dominance full size:", rec["mode"], n)
        adj = inputs.dominance_graph(n, fx["seed"])
        rows = torch.from_numpy(inputs.dense_to_rows(adj).view(np.int64)).to(DEV)
        mode = KZ_DOM_VERTEX if rec["mode"] == "vertex" else KZ_DOM_EDGE
        vm, em, res = kz.dominance(rows, mode)
        torch.cuda.synchronize()
        h = hashlib.sha256()
        h.update(vm.cpu().numpy().astype(np.uint8).tobytes())
        h.update(em.cpu().numpy().view(np.uint64).astype("<u8").tobytes())
        h.update(np.array([res["sweeps"], res["deleted_vertices"], res["deleted_edges"], res["events"]],
                          "<i8").tobytes())
        assert res["input_edges"] == rec["edges"], rec
        assert h.hexdigest() == rec["sha256"], (rec, res)
