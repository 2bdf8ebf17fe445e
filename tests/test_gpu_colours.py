"""More colour classes than the clique size on the GPU: the batched runtime
with a per-graph clique size (kz_batch_graph.clique, kz_request.clique)
against the oracle's O3 with the same thresholds (clique-1, clique-2; pinned
in tests/test_oracle.py).  Masks, rounds and exact-worklist counts are
equal, in every sharing mode, through the server, and bad clique sizes get
KZ_EINVAL."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import fixpoint_rows  # noqa: E402
from paper_2212_00574_amd import inputs  # noqa: E402
from paper_2212_00574_amd.binding import (Batch, BatchKernelizer, Kernelizer, Server,  # noqa: E402
                                          kz_batch_get_config, kz_batch_set_config)

DEV = torch.device("cuda", 0)


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def kz():
    k = Kernelizer(0)
    yield k
    k.close()


def graphs(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        m = int(rng.integers(3, 20))
        sizes = rng.integers(1, 140, size=m)
        g = inputs.make_graph(sizes, float(rng.uniform(0.15, 0.8)), seed=seed, gid=i,
                              plant=bool(rng.random() < 0.3), shuffle=False)
        rows, col, lay = g.bitset()
        clique = int(rng.integers(1, m + 1))
        out.append((rows, col, m, clique))
    return out


def check(b, res, gs, ctx):
    for i, (rows, col, m, clique) in enumerate(gs):
        ref = fixpoint_rows(rows, col, m, clique=clique)
        r = res[i]
        assert r["status"] == ref["status"] == 0, (ctx, i)
        assert r["rounds"] == ref["rounds"], (ctx, i, m, clique, int(r["rounds"]), ref["rounds"])
        assert r["surviving_vertices"] == ref["surv_vertices"], (ctx, i)
        assert r["surviving_edges"] == ref["surv_edges"], (ctx, i)
        assert r["edge_tests"] == ref["edge_tests"], (ctx, i)
        vm, em = b.masks(i)
        assert np.array_equal(vm, ref["vmask"]), (ctx, i)
        assert np.array_equal(em, ref["emask"]), (ctx, i)


@pytest.mark.parametrize("share", [0, 1, 2])
def test_batch_clique_below_classes_matches_oracle(kz, share):
    cfg0 = kz_batch_get_config(kz.ctx)
    try:
        kz_batch_set_config(kz.ctx, dict(cfg0, share=share))
        gs = graphs(20 + share, 48)
        say("colours: batch of", len(gs), "share", share)
        b = Batch(gs, DEV)
        BatchKernelizer(kz).run(b)
        torch.cuda.synchronize()
        check(b, b.read_results(), gs, share)
    finally:
        kz_batch_set_config(kz.ctx, cfg0)


def test_clique_equal_to_classes_is_the_plain_rule(kz):
    gs = [(r, c, m, m) for r, c, m, _ in graphs(30, 16)] + [(r, c, m, 0) for r, c, m, _ in graphs(31, 16)]
    b = Batch(gs, DEV)
    BatchKernelizer(kz).run(b)
    torch.cuda.synchronize()
    check(b, b.read_results(), [(r, c, m, m) for r, c, m, _ in gs], "clique = k")


def test_bad_clique_size_is_rejected(kz):
    rows, col, m, _ = graphs(40, 1)[0]
    b = Batch([(rows, col, m, m + 1), (rows, col, m, -2), (rows, col, m, 2)], DEV)
    BatchKernelizer(kz).run(b)
    torch.cuda.synchronize()
    res = b.read_results()
    assert res[0]["status"] == -1 and res[1]["status"] == -1 and res[2]["status"] == 0


def test_served_requests_with_a_clique_size(kz):
    gs = graphs(50, 24)
    srv = Server(kz, arena_bytes=256 << 20, max_slots=32)
    bufs, tickets = [], []
    for rows, col, m, clique in gs:
        r = torch.from_numpy(rows.view(np.int64)).to(DEV)
        c = torch.from_numpy(col).to(DEV)
        vm = torch.empty(col.size, dtype=torch.uint8, device=DEV)
        em = torch.empty_like(r)
        t = srv.submit(r, c, m, vm, em, clique)
        assert t is not None
        bufs.append((vm, em))
        tickets.append(t)
        srv.progress()
    t0 = time.time()
    out = [None] * len(gs)
    while any(o is None for o in out):
        for i, t in enumerate(tickets):
            if out[i] is None:
                out[i] = srv.poll(t)
        assert time.time() - t0 < 60
    for i, (rows, col, m, clique) in enumerate(gs):
        ref = fixpoint_rows(rows, col, m, clique=clique)
        assert out[i]["rounds"] == ref["rounds"] and out[i]["surviving_edges"] == ref["surv_edges"], i
        assert np.array_equal(bufs[i][0].cpu().numpy(), ref["vmask"]), i
        assert np.array_equal(bufs[i][1].cpu().numpy().view(np.uint64), ref["emask"]), i
    srv.close()
