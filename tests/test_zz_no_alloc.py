"""kz_kernelize_noalloc (the library's own workspace, no allocation) against
kz_kernelize (a caller's workspace) on the same inputs, through the C ABI:
two calls in a row, the second on a smaller graph, bit for bit; and a graph
larger than the fixed workspace is refused before any device work."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2212_00574_amd import inputs  # noqa: E402
from paper_2212_00574_amd.binding import (KZ_EWORKSPACE, NOALLOC_SCRATCH_BYTES, Kernelizer,  # noqa: E402
                                          _stream_handle, graph_bitset, graph_dense, kz_kernelize_noalloc,
                                          kz_workspace_bytes)

DEV = torch.device("cuda", 0)


def say(*a):
    print(*a, flush=True)


def run_both(kz, graph, colour, k, out_shape, out_dtype, n):
    ref_v = torch.full((n,), 7, dtype=torch.uint8, device=DEV)
    ref_e = torch.full(out_shape, 7, dtype=out_dtype, device=DEV)
    ref = kz.run(graph, colour, k, ref_v, ref_e)
    vm = torch.full((n,), 9, dtype=torch.uint8, device=DEV)
    em = torch.full(out_shape, 9, dtype=out_dtype, device=DEV)
    torch.cuda.synchronize()
    res = kz_kernelize_noalloc(kz.ctx, graph, colour.data_ptr(), k, vm.data_ptr(), em.data_ptr(),
                               _stream_handle(None, DEV)).as_dict()
    torch.cuda.synchronize()
    assert res["status"] == 0, res
    assert res == ref, (res, ref)
    assert torch.equal(vm, ref_v) and torch.equal(em, ref_e)
    return res


def test_noalloc_matches_kernelize_twice_second_smaller():
    kz = Kernelizer(0)
    try:
        # a bit-row graph of several blocks with ragged tails and a cascade
        big = inputs.make_graph([150, 97, 200, 64, 131, 75], 0.45, seed=11, gid=0, plant=True, shuffle=False)
        rows, col, lay = big.bitset()
        x = torch.from_numpy(rows.view(np.int64)).to(DEV)
        c = torch.from_numpy(col).to(DEV)
        g = graph_bitset(x)
        assert kz_workspace_bytes(kz.ctx, g, 6) <= NOALLOC_SCRATCH_BYTES
        say("noalloc call 1: bitset n=%d R=%d" % (x.shape[0], x.shape[1]))
        r1 = run_both(kz, g, c, 6, tuple(x.shape), torch.int64, x.shape[0])
        # second call: a smaller dense graph (caller vertex order)
        small = inputs.make_graph([20, 33, 17, 25], 0.5, seed=12, gid=1, plant=True)
        adj, colour = small.dense()
        a = torch.from_numpy(adj).to(DEV)
        c2 = torch.from_numpy(colour).to(DEV)
        say("noalloc call 2: dense n=%d" % a.shape[0])
        r2 = run_both(kz, graph_dense(a), c2, 4, tuple(a.shape), torch.uint8, a.shape[0])
        say("results", r1, r2)
    finally:
        kz.close()


def test_noalloc_refuses_a_graph_beyond_its_workspace():
    kz = Kernelizer(0)
    try:
        n, R = 24000, 400          # 77 MB of rows: its state copy alone is beyond 64 MiB
        x = torch.zeros((n, R), dtype=torch.int64, device=DEV)
        c = torch.zeros(n, dtype=torch.int32, device=DEV)
        g = graph_bitset(x)
        assert kz_workspace_bytes(kz.ctx, g, 20) > NOALLOC_SCRATCH_BYTES
        vm = torch.empty(n, dtype=torch.uint8, device=DEV)
        em = torch.empty_like(x)
        res = kz_kernelize_noalloc(kz.ctx, g, c.data_ptr(), 20, vm.data_ptr(), em.data_ptr(),
                                   _stream_handle(None, DEV))
        assert res.status == KZ_EWORKSPACE
    finally:
        kz.close()
