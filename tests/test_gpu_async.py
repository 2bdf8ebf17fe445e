"""The asynchronous single-graph call on the GPU: passes enqueued with no
host synchronisation, the result written by the device in stream order,
equal to the oracle in every format; continued one pass per call; input
errors reported through the result; and the whole call captured in a HIP
graph and replayed, every replay checked against the oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import kernelize_bitset, kernelize_csr, kernelize_dense  # noqa: E402
from paper_2212_00574_amd import inputs  # noqa: E402
from paper_2212_00574_amd.binding import (KZ_OUT_BYTES, Kernelizer, KzError, graph_bitset,  # noqa: E402
                                          graph_csr, graph_dense, kz_out_from_bytes)

DEV = torch.device("cuda", 0)


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def kz():
    k = Kernelizer(0)
    yield k
    k.close()


def read_out(out):
    torch.cuda.synchronize()
    return kz_out_from_bytes(out.cpu().numpy().tobytes())


def check(o, ref, vm, em, ctx):
    assert o["status"] == 0 and ref["status"] == 0, ctx
    assert o["converged"] == 1, ctx
    assert o["rounds"] == ref["rounds"] and o["equals_input"] == ref["equals_input"], ctx
    assert o["passes"] == ref["rounds"] + 1, ctx
    assert o["surviving_vertices"] == ref["surv_vertices"], ctx
    assert o["surviving_edges"] == ref["surv_edges"], ctx
    assert o["edge_tests"] == ref["edge_tests"], ctx
    assert np.array_equal(vm, ref["vmask"]), ctx
    assert np.array_equal(em, ref["emask"]), ctx


class Case:
    """One seeded graph in the three input formats, with device buffers."""

    def __init__(self, sizes, p, gid, plant=True):
        g = inputs.make_graph(sizes, p, seed=61, gid=gid, plant=plant, shuffle=False)
        self.k = len(sizes)
        self.adj, self.colour = g.dense()
        self.rows, self.scol, lay = g.bitset()
        self.rp, self.ci = inputs.dense_to_csr(self.adj)
        self.n, self.R = lay.n, lay.R

    def buffers(self, fmt):
        n = self.n
        if fmt == "dense":
            adj = torch.from_numpy(self.adj).to(DEV)
            return (graph_dense(adj), torch.from_numpy(self.colour).to(DEV), adj,
                    torch.empty(n, dtype=torch.uint8, device=DEV), torch.empty((n, n), dtype=torch.uint8, device=DEV))
        if fmt == "bitset":
            rows = torch.from_numpy(self.rows.view(np.int64)).to(DEV)
            return (graph_bitset(rows), torch.from_numpy(self.scol).to(DEV), rows,
                    torch.empty(n, dtype=torch.uint8, device=DEV), torch.empty_like(rows))
        rp = torch.from_numpy(self.rp).to(DEV)
        ci = torch.from_numpy(self.ci).to(DEV)
        return (graph_csr(rp, ci), torch.from_numpy(self.colour).to(DEV), (rp, ci),
                torch.empty(n, dtype=torch.uint8, device=DEV), torch.empty(len(self.ci), dtype=torch.uint8, device=DEV))

    def oracle(self, fmt):
        if fmt == "dense":
            return kernelize_dense(self.adj, self.colour, self.k)
        if fmt == "bitset":
            return kernelize_bitset(self.rows, self.scol, self.k)
        return kernelize_csr(self.rp, self.ci, self.colour, self.k)

    def masks(self, fmt, vm, em):
        torch.cuda.synchronize()
        v = vm.cpu().numpy()
        e = em.cpu().numpy()
        return v, (e.view(np.uint64) if fmt == "bitset" else e)


CASES = [([30, 25, 40, 35], 0.45, 0), ([60] * 6, 0.3, 1), ([20, 90, 70, 15, 64, 33], 0.25, 2),
         ([128, 128, 128], 0.2, 3)]
FORMATS = ("dense", "bitset", "csr")


def test_async_one_call_equals_oracle(kz):
    for sizes, p, gid in CASES:
        c = Case(sizes, p, gid)
        for fmt in FORMATS:
            say("async one call", fmt, sizes, p)
            graph, colour, _keep, vm, em = c.buffers(fmt)
            out = torch.zeros(KZ_OUT_BYTES, dtype=torch.uint8, device=DEV)
            kz.run_async(graph, colour, c.k, vm, em, out, first_pass=1, npasses=64)
            o = read_out(out)
            ref = c.oracle(fmt)
            v, e = c.masks(fmt, vm, em)
            check(o, ref, v, e, (fmt, sizes))
            # the blocking call (chunks of the same passes) agrees
            vm2, em2 = torch.empty_like(vm), torch.empty_like(em)
            res = kz.run(graph, colour, c.k, vm2, em2)
            assert {key: res[key] for key in res} == {key: o[key] for key in res}, (fmt, sizes)
            v2, e2 = c.masks(fmt, vm2, em2)
            assert np.array_equal(v2, v) and np.array_equal(e2, e), (fmt, sizes)


def test_async_one_pass_per_call(kz):
    """Continuing a run one pass per call reaches the same fixpoint; before
    it, the result counts the passes so far and is not converged."""
    c = Case([60] * 6, 0.3, 1)
    for fmt in FORMATS:
        say("async one pass per call", fmt)
        graph, colour, _keep, vm, em = c.buffers(fmt)
        out = torch.zeros(KZ_OUT_BYTES, dtype=torch.uint8, device=DEV)
        ws = None
        calls = 0
        while True:
            calls += 1
            ws = kz.run_async(graph, colour, c.k, vm, em, out, first_pass=calls, npasses=1, ws=ws)
            o = read_out(out)
            assert o["passes"] == calls, (fmt, calls)
            if o["converged"]:
                break
            assert o["rounds"] == calls and calls < 200, (fmt, calls)
        ref = c.oracle(fmt)
        v, e = c.masks(fmt, vm, em)
        check(o, ref, v, e, fmt)
        assert calls == ref["rounds"] + 1
        # passes enqueued past the fixpoint do nothing and change nothing
        kz.run_async(graph, colour, c.k, vm, em, out, first_pass=calls + 1, npasses=3, ws=ws)
        o2 = read_out(out)
        assert o2 == o, fmt
        v2, e2 = c.masks(fmt, vm, em)
        assert np.array_equal(v2, v) and np.array_equal(e2, e), fmt


def test_async_errors(kz):
    c = Case([20, 20, 20], 0.5, 4, plant=False)
    bad = c.colour.copy()
    bad[3] = 7                                      # colour outside [0, k)
    adj = torch.from_numpy(c.adj).to(DEV)
    out = torch.zeros(KZ_OUT_BYTES, dtype=torch.uint8, device=DEV)
    vm = torch.empty(c.n, dtype=torch.uint8, device=DEV)
    em = torch.empty((c.n, c.n), dtype=torch.uint8, device=DEV)
    bad_t = torch.from_numpy(bad).to(DEV)
    kz.run_async(graph_dense(adj), bad_t, c.k, vm, em, out, npasses=4)
    o = read_out(out)
    assert o["status"] == -2 and o["converged"] == 1
    ill = c.adj.copy()
    ill[0, 1] = ill[1, 0] = 1                       # an edge inside class 0
    ill_t = torch.from_numpy(ill).to(DEV)           # held: the call does not wait for its kernels
    col_t = torch.from_numpy(c.colour).to(DEV)
    kz.run_async(graph_dense(ill_t), col_t, c.k, vm, em, out, npasses=4)
    o = read_out(out)
    assert o["status"] == -3 and o["converged"] == 1
    with pytest.raises(KzError):                    # host-detectable: nothing enqueued
        kz.run_async(graph_dense(adj), torch.from_numpy(c.colour).to(DEV), c.k, vm, em, out, npasses=0)
    empty = torch.empty((0, 0), dtype=torch.uint8, device=DEV)
    none = torch.empty(0, dtype=torch.int32, device=DEV)
    kz.run_async(graph_dense(empty), none, 3, vm, em, out, npasses=2)
    o = read_out(out)
    assert o["status"] == 0 and o["converged"] == 1 and o["equals_input"] == 1


def test_async_captured_in_hip_graph(kz):
    """The call captured once and replayed: every replay, after eager work
    has overwritten the outputs, equals the oracle."""
    for sizes, p, gid in CASES[1:3]:
        c = Case(sizes, p, gid)
        for fmt in FORMATS:
            say("async captured", fmt, sizes, p)
            graph, colour, _keep, vm, em = c.buffers(fmt)
            out = torch.zeros(KZ_OUT_BYTES, dtype=torch.uint8, device=DEV)
            ws = kz.workspace(graph, c.k)
            ref = c.oracle(fmt)
            npasses = ref["rounds"] + 4
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):           # one eager run before the capture
                kz.run_async(graph, colour, c.k, vm, em, out, npasses=npasses, ws=ws,
                             stream=torch.cuda.current_stream())
            torch.cuda.current_stream().wait_stream(side)
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                kz.run_async(graph, colour, c.k, vm, em, out, npasses=npasses, ws=ws,
                             stream=torch.cuda.current_stream())
            for rep in range(3):
                vm.fill_(7)
                em.fill_(5)
                out.zero_()
                torch.cuda.synchronize()
                g.replay()
                o = read_out(out)
                v, e = c.masks(fmt, vm, em)
                check(o, ref, v, e, (fmt, sizes, "replay", rep))
            del g
