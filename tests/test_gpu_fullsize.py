"""Full-size parity with the CPU oracle, in the launch configurations the
benchmark times: the whole config-3a graph (bit-row witness path, int8 MFMA
path and the no-allocation call), all 4096 graphs of the batching workload
(autotuned, one persistent launch) and the covered requests of the serving
workload (every request with n <= 5000, a seeded 2% of the others and the
100 largest, served in a mix).  The expected values are SHA-256 digests of
each graph's (vmask || emask || rounds, survivors, edge tests) written by
tests/golden/make_golden.py from the oracle (O3, pinned against O1); inputs
are materialised on the device by kz_gen_bitset, which tests/test_gpu_gen.py
checks bit for bit against the Python generator the oracle's inputs come
from."""
import hashlib
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2212_00574_amd import inputs  # noqa: E402
from paper_2212_00574_amd.binding import (KZ_EDGE_BITSET, KZ_EDGE_MFMA_I8, Batch, BatchKernelizer,  # noqa: E402
                                          Kernelizer, Server, _stream_handle, graph_bitset, kz_gen_bitset,
                                          kz_kernelize_noalloc)

DEV = torch.device("cuda", 0)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)


def golden(name):
    return json.load(open(os.path.join(GOLDEN, name)))


def digest(vmask, emask, r):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(vmask, np.uint8).tobytes())
    h.update(np.ascontiguousarray(emask).view(np.uint64).astype("<u8", copy=False).tobytes())
    h.update(np.array([r["rounds"], r["surviving_vertices"], r["surviving_edges"], r["edge_tests"]],
                      "<i8").tobytes())
    return h.digest()


@pytest.fixture(scope="module")
def kz():
    k = Kernelizer(0)
    yield k
    k.close()


def gen_graph(kz, sizes, p, seed, gid, planted=None):
    lay = inputs.class_layout(sizes)
    rows = torch.empty((lay.n, lay.R), dtype=torch.int64, device=DEV)
    colour = torch.empty(lay.n, dtype=torch.int32, device=DEV)
    kz_gen_bitset(kz.ctx, sizes, p, seed, gid, planted, rows.data_ptr(), lay.R, colour.data_ptr(), None)
    return rows, colour


@pytest.mark.parametrize("path", ["bitset", "mfma", "noalloc"])
def test_config3a_whole_graph_matches_oracle(kz, path):
    g = golden("c3a_seed0.json")
    rows, colour = gen_graph(kz, [1000] * 20, 0.3, 0, 0)
    vm = torch.empty(rows.shape[0], dtype=torch.uint8, device=DEV)
    em = torch.empty_like(rows)
    say("c3a", path, "n=%d R=%d" % tuple(rows.shape))
    if path == "noalloc":
        res = kz_kernelize_noalloc(kz.ctx, graph_bitset(rows), colour.data_ptr(), 20, vm.data_ptr(), em.data_ptr(),
                                   _stream_handle(None, DEV)).as_dict()
    else:
        kz.set_edge_path(KZ_EDGE_MFMA_I8 if path == "mfma" else KZ_EDGE_BITSET)
        try:
            res = kz.run(graph_bitset(rows), colour, 20, vm, em)
        finally:
            kz.set_edge_path(KZ_EDGE_BITSET)
    torch.cuda.synchronize()
    assert res["status"] == 0
    for key in ("rounds", "edge_tests"):
        assert res[key] == g[key], key
    assert res["surviving_vertices"] == g["surv_vertices"] and res["surviving_edges"] == g["surv_edges"]
    assert digest(vm.cpu().numpy(), em.cpu().numpy(), res).hex() == g["sha256"]


def bucket_hashes(digests, ids, size):
    out = []
    for b0 in range(0, len(ids), size):
        h = hashlib.sha256()
        for i in ids[b0:b0 + size]:
            h.update(digests[i])
        out.append(h.hexdigest())
    return out


def test_config4_all_4096_graphs_match_oracle(kz):
    g = golden("c4_seed0.json")
    specs = inputs.config4_specs(0)
    shapes = [(int(sp.sizes.sum()), int(((sp.sizes + 63) // 64).sum()), sp.k) for sp in specs]
    b = Batch.allocate(shapes, DEV)
    say("c4: materialising %d graphs" % b.G)
    for i, sp in enumerate(specs):
        d = b.desc[i]
        n, R = int(d["n"]), int(d["row_words"])
        a, o = int(d["row_offset"]), int(d["vertex_offset"])
        planted = inputs.config4_graph(sp, 0, i).planted
        kz_gen_bitset(kz.ctx, sp.sizes, sp.p, 0, i, planted, b.rows[a:].data_ptr(), R, b.colour[o:].data_ptr(), None)
    bk = BatchKernelizer(kz)
    say("c4: autotune and run")
    bk.autotune(b)
    bk.run(b)
    torch.cuda.synchronize()
    res = b.read_results()
    assert np.all(res["status"] == 0)
    vm_all = b.vmask.cpu().numpy()
    em_all = b.emask.cpu().numpy()
    digests = {}
    for i in range(b.G):
        d = b.desc[i]
        n, R = int(d["n"]), int(d["row_words"])
        a, o = int(d["row_offset"]), int(d["vertex_offset"])
        r = {k: int(res[i][k]) for k in ("rounds", "surviving_vertices", "surviving_edges", "edge_tests")}
        digests[i] = digest(vm_all[o:o + n], em_all[a:a + n * R], r)
    got = bucket_hashes(digests, list(range(b.G)), g["bucket"])
    for j, bk_ in enumerate(g["buckets"]):
        lo, hi = bk_["ids"]
        sl = res[lo:hi + 1]
        assert int(sl["rounds"].sum()) == bk_["rounds"] and int(sl["edge_tests"].sum()) == bk_["edge_tests"], j
        assert got[j] == bk_["hash"], ("bucket", j, lo, hi)


C5_PARTS = 4


@pytest.mark.parametrize("part", range(C5_PARTS))
def test_config5_covered_requests_match_oracle_in_a_mix(kz, part):
    """One quarter of the covered buckets, served together in a mix."""
    g = golden("c5_seed0.json")
    specs = inputs.config5_specs(0)
    buckets = g["buckets"][part::C5_PARTS]
    ids = [i for b_ in buckets for i in b_["ids"]]
    say("c5 part %d: %d requests in %d buckets" % (part, len(ids), len(buckets)))
    srv = Server(kz, arena_bytes=16 << 30, max_slots=1024)
    digests, pending, done = {}, [], 0
    queue = list(ids)
    live = {}
    try:
        while queue or live:
            while queue:
                i = queue[0]
                sp = specs[i]
                lay = inputs.class_layout(sp.sizes)
                if i not in live:
                    rows = torch.empty((lay.n, lay.R), dtype=torch.int64, device=DEV)
                    colour = torch.empty(lay.n, dtype=torch.int32, device=DEV)
                    kz_gen_bitset(kz.ctx, sp.sizes, sp.p, 0, i, None, rows.data_ptr(), lay.R, colour.data_ptr(),
                                  srv.stream.cuda_stream)
                    vm = torch.empty(lay.n, dtype=torch.uint8, device=DEV)
                    em = torch.empty_like(rows)
                    live[i] = (rows, colour, vm, em, None)
                rows, colour, vm, em, _ = live[i]
                t = srv.submit(rows, colour, sp.k, vm, em)
                if t is None:
                    break
                live[i] = (rows, colour, vm, em, t)
                queue.pop(0)
            srv.progress()
            for i in list(live):
                rows, colour, vm, em, t = live[i]
                if t is None:
                    continue
                r = srv.poll(t)
                if r is None:
                    continue
                assert r["status"] == 0, (i, r)
                torch.cuda.synchronize()
                digests[i] = digest(vm.cpu().numpy(), em.cpu().numpy(), r)
                del live[i]
                done += 1
                if done % 2000 == 0:
                    say("c5 part %d: %d done" % (part, done))
    finally:
        srv.close()
    for b_ in buckets:
        h = hashlib.sha256()
        for i in b_["ids"]:
            h.update(digests[i])
        assert h.hexdigest() == b_["hash"], ("bucket from request", b_["ids"][0])
