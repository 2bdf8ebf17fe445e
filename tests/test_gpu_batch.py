"""Batched path on the GPU: every graph of a mixed batch must match the oracle
and the single-graph path bit for bit, also under hipGraph replay and after
autotuning."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import kernelize_bitset  # noqa: E402
from paper_2212_00574_amd import inputs  # noqa: E402
from paper_2212_00574_amd.binding import (KZ_ETOOLARGE, Batch, BatchKernelizer, Kernelizer,  # noqa: E402
                                          kz_batch_get_config, kz_batch_set_config)

DEV = torch.device("cuda", 0)


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def kz():
    k = Kernelizer(0)
    yield k
    k.close()


def mixed_graphs(count, seed, small=False):
    """Graphs shaped like the batching workload (scaled down when small)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        k = int(rng.integers(3 if small else 4, 9 if small else 17))
        hi = 40 if small else 129
        sizes = rng.integers(1 if small else 8, hi, size=k)
        p = float(rng.uniform(0.2, 0.8))
        g = inputs.make_graph(sizes, p, seed=seed, gid=i, plant=bool(rng.random() < 0.1), shuffle=False)
        rows, col, lay = g.bitset()
        out.append((rows, col, k))
    return out


def check_batch(kz, graphs, ctx, bk=None):
    say("batch", ctx, len(graphs), "graphs")
    b = Batch(graphs, DEV)
    bk = bk or BatchKernelizer(kz)
    bk.run(b)
    torch.cuda.synchronize()
    res = b.read_results()
    for i, (rows, col, k) in enumerate(graphs):
        ref = kernelize_bitset(rows, col, k)
        r = res[i]
        assert r["status"] == ref["status"], (ctx, i, r["status"], ref["status"])
        if ref["status"]:
            continue
        if r["rounds"] != ref["rounds"]:
            vm, em = b.masks(i)
            detail = {"rounds": (int(r["rounds"]), ref["rounds"]),
                      "surv_v": (int(r["surviving_vertices"]), ref["surv_vertices"]),
                      "surv_e": (int(r["surviving_edges"]), ref["surv_edges"]),
                      "tests": (int(r["edge_tests"]), ref["edge_tests"]),
                      "vmask_equal": bool(np.array_equal(vm, ref["vmask"])),
                      "emask_equal": bool(np.array_equal(em, ref["emask"]))}
            raise AssertionError("%s graph %d: %s" % (ctx, i, detail))
        assert r["rounds"] == ref["rounds"] and r["equals_input"] == ref["equals_input"], (ctx, i)
        assert r["surviving_vertices"] == ref["surv_vertices"], (ctx, i)
        assert r["surviving_edges"] == ref["surv_edges"], (ctx, i)
        assert r["edge_tests"] == ref["edge_tests"], (ctx, i)
        vm, em = b.masks(i)
        assert np.array_equal(vm, ref["vmask"]), (ctx, i)
        assert np.array_equal(em, ref["emask"]), (ctx, i)
    return b, res


def test_batch_matches_oracle(kz):
    check_batch(kz, mixed_graphs(48, seed=1, small=True), "small")


def test_batch_matches_oracle_workload_shape(kz):
    check_batch(kz, mixed_graphs(24, seed=2), "shape")


def test_batch_edge_cases_and_errors(kz):
    graphs = []
    for sizes, p in [([5, 7, 9], 0.0), ([30], 0.0), ([20, 25], 0.1), ([64, 64, 65], 0.5), ([3, 0, 4, 5], 0.7),
                     ([12] * 9, 0.6)]:
        g = inputs.make_graph(sizes, p, seed=3, gid=len(graphs), shuffle=False)
        rows, col, lay = g.bitset()
        graphs.append((rows, col, len(sizes)))
    # illegal input: a self-loop and an asymmetric pair
    rows, col, k = graphs[3]
    bad = rows.copy(); bad[2, 0] |= np.uint64(1 << 2)
    graphs.append((bad, col, k))
    bad = rows.copy(); bad[70, 0] ^= np.uint64(1 << 9)
    graphs.append((bad, col, k))
    # colour out of range, unsorted colours
    bad_col = col.copy(); bad_col[-1] = k + 1
    graphs.append((rows, bad_col, k))
    graphs.append((rows, col[::-1].copy(), k))
    check_batch(kz, graphs, "edge-cases")


def test_batch_too_large_graph_is_flagged(kz):
    small = mixed_graphs(3, seed=4, small=True)
    big = inputs.make_graph([1] * 65, 0.5, seed=4, gid=9, shuffle=False)   # k = 65 > batch limit
    rows, col, lay = big.bitset()
    b = Batch(small + [(rows, col, 65)], DEV)
    BatchKernelizer(kz).run(b)
    torch.cuda.synchronize()
    res = b.read_results()
    assert res[3]["status"] == KZ_ETOOLARGE
    assert all(res[i]["status"] == 0 for i in range(3))


def test_batch_matches_single_graph_path(kz):
    graphs = mixed_graphs(16, seed=5)
    b, res = check_batch(kz, graphs, "vs-single")
    for i, (rows, col, k) in enumerate(graphs):
        vm, em, r = kz.kernelize_bitset(torch.from_numpy(rows.view(np.int64)).to(DEV),
                                        torch.from_numpy(col).to(DEV), k)
        torch.cuda.synchronize()
        bvm, bem = b.masks(i)
        assert np.array_equal(vm.cpu().numpy(), bvm)
        assert np.array_equal(em.cpu().numpy().view(np.uint64), bem)
        assert r["rounds"] == res[i]["rounds"] and r["edge_tests"] == res[i]["edge_tests"]


def test_batch_hipgraph_replay(kz):
    """Capture the batch once and replay it; every replay must reproduce the eager result."""
    graphs = mixed_graphs(32, seed=6, small=True)
    b = Batch(graphs, DEV)
    bk = BatchKernelizer(kz)
    bk.run(b)
    torch.cuda.synchronize()
    eager_res = b.read_results().copy()
    eager_v = b.vmask.clone()
    eager_e = b.emask.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bk.run(b, stream=side)   # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        bk.run(b)
    for rep in range(4):
        b.vmask.fill_(7)
        b.emask.fill_(0)
        b.results.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        # the graphs' ranges (the padding between them is nobody's output)
        for i in range(b.G):
            d = b.desc[i]
            n, R = int(d["n"]), int(d["row_words"])
            a, o = int(d["row_offset"]), int(d["vertex_offset"])
            assert torch.equal(b.vmask[o:o + n], eager_v[o:o + n]), (rep, i)
            assert torch.equal(b.emask[a:a + n * R], eager_e[a:a + n * R]), (rep, i)
        assert np.array_equal(b.read_results(), eager_res), rep


def test_batch_autotune_keeps_results(kz):
    graphs = mixed_graphs(40, seed=7, small=True)
    b = Batch(graphs, DEV)
    bk = BatchKernelizer(kz)
    before = kz_batch_get_config(kz.ctx)
    best = bk.autotune(b)
    assert best["waves"] in (4, 8, 16) and best["chunk"] in (4, 8)
    assert kz_batch_get_config(kz.ctx) == best
    check_batch(kz, graphs, "tuned", bk)
    for cfg in ({"waves": 4, "chunk": 4, "lpt": 0, "workgroups": 3}, {"waves": 16, "chunk": 4, "lpt": 1,
                                                                       "workgroups": 0},
                {"waves": 8, "chunk": 8, "lpt": 1, "workgroups": 17}):
        kz_batch_set_config(kz.ctx, cfg)
        check_batch(kz, graphs, "cfg%s" % cfg, bk)
    with pytest.raises(Exception):
        kz_batch_set_config(kz.ctx, {"waves": 16, "chunk": 8, "lpt": 1, "workgroups": 0})
    kz_batch_set_config(kz.ctx, before)


def cascade_graphs():
    """Three graphs of the batching workload whose fixpoints take 28 to 77
    rounds (seed 0, ids 0, 2826, 4063), among small ones: once the queue is
    empty their passes are shared with the idle workgroups."""
    specs = inputs.config4_specs(0, graphs=4096)
    heavy = []
    for gid in (4063, 2826, 0):
        rows, col, lay = inputs.config4_graph(specs[gid], 0, gid).bitset()
        heavy.append((rows, col, specs[gid].k))
    return heavy + mixed_graphs(24, seed=8, small=True)


@pytest.mark.parametrize("share", [0, 1, 2])
def test_batch_share_modes(kz, share):
    """Passes shared across workgroups (also every pass, share=1) or kept by
    one workgroup (share=2) give the same masks, rounds and counts."""
    graphs = mixed_graphs(40, seed=9, small=True) + mixed_graphs(8, seed=10)
    before = kz_batch_get_config(kz.ctx)
    try:
        for waves, chunk in ((8, 8), (16, 4), (4, 4)):
            kz_batch_set_config(kz.ctx, {"waves": waves, "chunk": chunk, "lpt": 1, "workgroups": 0, "share": share})
            check_batch(kz, graphs, "share%d-%dx%d" % (share, waves, chunk))
    finally:
        kz_batch_set_config(kz.ctx, before)


@pytest.mark.parametrize("share", [0, 1])
def test_batch_cascades_with_helpers(kz, share):
    before = kz_batch_get_config(kz.ctx)
    try:
        kz_batch_set_config(kz.ctx, {"waves": 8, "chunk": 8, "lpt": 1, "workgroups": 0, "share": share})
        b, res = check_batch(kz, cascade_graphs(), "cascades-share%d" % share)
        assert min(int(res[i]["rounds"]) for i in range(3)) >= 28
    finally:
        kz_batch_set_config(kz.ctx, before)


def test_batch_large_graphs(kz):
    """Graphs beyond 4096 vertices and 128 row words (up to the path's
    32768 / 512 limits) next to small ones; their passes are shared."""
    graphs = []
    for gid, (sizes, p) in ((0, ([700] * 8, 0.06)), (3, ([2100] * 4, 0.05))):   # 4-round cascades, R = 88 / 132
        g = inputs.make_graph(sizes, p, seed=12, gid=gid, plant=True, shuffle=False)
        rows, col, lay = g.bitset()
        graphs.append((rows, col, len(sizes)))
    check_batch(kz, graphs + mixed_graphs(12, seed=13, small=True), "large")
