"""Benchmark: colour-index kernelization to the fixpoint on one MI355X.

A step is one full kz_kernelize call (validation, every pass to the fixpoint,
outputs) on inputs already resident in device memory.  The default workload
is the mid-size graph: k = 10 colour classes x 300 vertices, inter-class edge
probability 0.6, one planted 10-clique, class-major uint64 bit rows.

Prints one JSON line.  ``value`` is edge tests per second, counting the
edge tests of the exact worklists (every edge in the first pass; in pass r+1
the edges with an endpoint that lost an edge in round r).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0           # MI355X HBM3E, published
I8_PEAK_TOPS = 5000.0            # MI355X dense int8 MFMA, published (no sparsity)
# 32-bit integer VALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one wave64
# instruction per SIMD every 4 clocks); bitwise ops have no packed form.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

WORKLOADS = {
    "c1": "k=4 classes x 25 vertices (n=100), p=0.5, dense uint8 input",
    "c2": "k=10 classes x 300 vertices (n=3000), p=0.6, planted 10-clique, uint64 bit rows",
    "c3a": "k=20 classes x 1000 vertices (n=20000), p=0.3, uint64 bit rows",
    "c3b": "k=30 multinomial classes, n=100000, 2.5M uniform inter-class edges (avg degree 50), CSR",
    "c4": "4096 graphs, k~U{4..16}, class sizes~U{8..128}, p~U[0.2,0.8], 10% planted k-clique, uint64 bit rows",
    "c5": "served requests: n log-uniform [200,20000], k~U{5..30} near-equal classes, p~U[0.1,0.9], Poisson "
          "arrivals, uint64 bit rows materialised on the device at arrival",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-one-by-one", action="store_true",
                    help="c4: skip the one-graph-at-a-time comparison (for counter runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=None,
                    help="steps of the per-kernel event-timed loop (default: --steps)")
    ap.add_argument("--edge-path", default="bitset", choices=("bitset", "mfma"),
                    help="edge test of the single-graph path: witness search on bit rows, or int8 MFMA counts")
    ap.add_argument("--requests", type=int, default=2000,
                    help="c5: requests per phase (a bounded prefix of the 50k-request stream)")
    ap.add_argument("--copy-calibration", type=int, default=None, metavar="MIB",
                    help="only run device-to-device copies of MIB MiB (memory-counter calibration)")
    return ap.parse_args()


def make_workload(name, seed):
    from paper_2212_00574_amd import inputs
    if name == "c1":
        g = inputs.config1(seed)
        adj, colour = g.dense()
        return dict(fmt="dense", adj=adj, colour=colour, k=4, sizes=g.sizes, graph=g)
    if name == "c3b":
        sg = inputs.config3b(seed)
        return dict(fmt="csr", rp=sg.row_ptr, ci=sg.col_idx, colour=sg.colour, k=sg.k, sizes=sg.sizes, graph=sg)
    g = inputs.config2(seed) if name == "c2" else inputs.config3a(seed)
    rows, colour, lay = g.bitset()
    return dict(fmt="bitset", rows=rows, colour=colour, k=g.k, sizes=g.sizes, layout=lay, graph=g)


def pair_edge_counts(w):
    """Edges between every pair of classes (from the generated input, CPU side)."""
    from paper_2212_00574_amd import inputs
    g = w["graph"]
    lay = inputs.class_layout(g.sizes)
    k = lay.k
    cnt = np.zeros((k, k), np.int64)
    slot = g.dense_slot() if g.n <= 6000 else None
    for a in range(k):
        if slot is not None:
            blk = slot[lay.offsets[a]:lay.offsets[a + 1]]
        else:
            blk = g.slot_rows(int(lay.offsets[a]), int(lay.offsets[a + 1]))
        for b in range(k):
            cnt[a, b] = int(blk[:, lay.offsets[b]:lay.offsets[b + 1]].sum())
    return cnt


def csr_operand_bytes(w):
    """Sum over edges of 4 (deg u + deg v): the two rows a merge-based test reads."""
    deg = np.diff(w["rp"]).astype(np.int64)
    src = np.repeat(np.arange(len(deg)), deg)
    up = src < w["ci"]
    return float(4 * (deg[src[up]] + deg[w["ci"][up]]).sum()), int(up.sum())


def edge_work(w):
    """Per-edge figures of the edge test, summed over all edges of the input.

    operand bytes: 2 (n - s_cu - s_cv) / 8 -- both rows minus the endpoints'
    own classes, i.e. what a test that streams the rows reads;
    algorithmic ops: for every third class c, W_c = ceil(s_c/64) words, each
    one AND and one OR-accumulate on two 32-bit halves (4 ops per word).
    """
    sizes = np.asarray(w["sizes"], np.int64)
    n = int(sizes.sum())
    words = (sizes + 63) // 64
    R = int(words.sum())
    cnt = pair_edge_counts(w)
    k = len(sizes)
    op_bytes, ops = 0, 0
    for a in range(k):
        for b in range(a + 1, k):
            m_ab = int(cnt[a, b])
            op_bytes += m_ab * 2 * (n - sizes[a] - sizes[b]) / 8
            ops += m_ab * 4 * (R - words[a] - words[b])
    return float(op_bytes), float(ops), int(np.triu(cnt, 1).sum())


# The kernel whose launches set each workload's roofline, and the sources it
# is built from (a committed counter summary is used only while they match).
PROFILED = {
    "c1": ("k_edge", ("kz_kernels.hip", "kz_internal.h")),
    "c2": ("k_edge", ("kz_kernels.hip", "kz_internal.h")),
    "c3a": ("k_edge", ("kz_kernels.hip", "kz_internal.h")),
    "c3b": ("k_csr_edge", ("kz_csr.hip", "kz_internal.h")),
    "c4": ("k_batch", ("kz_batch.hip", "kz_internal.h")),
}


def _code_only(text):
    """Source text without comments and with whitespace collapsed (the
    sources hold no comment markers inside string literals)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def source_hash(workload="c2"):
    """Hash of the code (comments and layout ignored) the workload's roofline
    kernel is built from."""
    h = hashlib.sha256()
    for f in PROFILED.get(workload, PROFILED["c2"])[1]:
        h.update(_code_only(open(os.path.join(ROOT, "paper_2212_00574_amd", "csrc", f)).read()).encode())
    return h.hexdigest()[:16]


def profile_value(workload, key):
    """A figure ("- key: value") of the committed counter summary
    profiles/<kernel>_<workload>.md of the workload's roofline kernel; None
    when absent or when the kernel's sources changed since the counters were
    taken ("- source_sha: S")."""
    kernel = PROFILED.get(workload, PROFILED["c2"])[0]
    path = os.path.join(ROOT, "profiles", "%s_%s.md" % (kernel, workload))
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        line = line.strip()
        if line.startswith("- ") and ":" in line:
            k, val = line[2:].split(":", 1)
            vals[k.strip()] = val.strip()
    if vals.get("source_sha") != source_hash(workload) or key not in vals:
        return None
    try:
        return float(vals[key])
    except ValueError:
        return None


def traffic_from_profile(workload):
    """HBM bytes per launch of the workload's roofline kernel (FETCH_SIZE and
    WRITE_SIZE, scaled by a plain copy's readings)."""
    return profile_value(workload, "hbm_bytes_per_launch")


# What the full-segment models leave out (the ops and bytes that the
# roofline's "achieved" counts are fixed per test, whatever a kernel does).
ALU_MODEL_NOTE = ("achieved/frac count the full-segment test's ops (AND + OR per word of both rows in every third "
                  "class); the witness search stops at the first word with a common neighbour, so it issues fewer "
                  "ops than the model and frac can pass 1. valu_issue_frac is the VALU lane-ops the kernel actually "
                  "issued (SQ_INSTS_VALU x 64 per launch, committed counter summary) over the same peak.")
CSR_MODEL_NOTE = ("achieved/frac count both rows' int32 entries for every tested edge; the rows of a 100000-vertex "
                  "graph are re-read from L2 and the Infinity Cache, so this stream can pass the HBM peak. traffic "
                  "is the counter-measured HBM bytes per launch; the kernel is bound by gather latency, not HBM.")


def cpu_baseline(w):
    from oracle import FMT_BITSET, FMT_CSR, FMT_DENSE, OracleGraph
    t0 = time.perf_counter()
    if w["fmt"] == "dense":
        g = OracleGraph(FMT_DENSE, len(w["colour"]), w["k"], w["colour"], adj=w["adj"])
    elif w["fmt"] == "csr":
        g = OracleGraph(FMT_CSR, len(w["colour"]), w["k"], w["colour"], row_ptr=w["rp"], col_idx=w["ci"])
    else:
        g = OracleGraph(FMT_BITSET, len(w["colour"]), w["k"], w["colour"], rows=w["rows"],
                        row_words=w["rows"].shape[1])
    t1 = time.perf_counter()
    res = g.fixpoint()
    t2 = time.perf_counter()
    vm, em = g.masks()
    return res, (vm, em), t2 - t1, t1 - t0


def _gen_c4(args):
    from paper_2212_00574_amd import inputs
    spec, seed, gid = args
    rows, colour, lay = inputs.config4_graph(spec, seed, gid).bitset()
    return rows, colour, spec.k


def c4_graphs(seed, count=4096, procs=16):
    """The batching workload, generated in worker processes (before any GPU use)."""
    import multiprocessing as mp
    from paper_2212_00574_amd import inputs
    specs = inputs.config4_specs(seed, graphs=count)
    with mp.get_context("fork").Pool(procs) as pool:
        return pool.map(_gen_c4, [(sp, seed, i) for i, sp in enumerate(specs)], chunksize=32)


def bench_batch(args):
    """Config 4: batched graphs/s against one-graph-at-a-time launches."""
    t0 = time.perf_counter()
    graphs = c4_graphs(args.seed)
    gen_s = time.perf_counter() - t0
    print("generated %d graphs in %.1f s" % (len(graphs), gen_s), file=sys.stderr, flush=True)
    import torch

    from paper_2212_00574_amd.binding import Batch, BatchKernelizer, Kernelizer, graph_bitset
    dev = torch.device("cuda", 0)
    kz = Kernelizer(0)
    b = Batch(graphs, dev)
    bk = BatchKernelizer(kz)
    tuned = bk.autotune(b)
    bk.run(b)
    torch.cuda.synchronize()
    res = b.read_results()
    assert np.all(res["status"] == 0), np.unique(res["status"])
    # capture once, replay in the timed loop
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bk.run(b, stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    tc0 = time.perf_counter()
    with torch.cuda.graph(graph):
        bk.run(b)
    capture_ms = (time.perf_counter() - tc0) * 1e3
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    kernel_ms = e0.elapsed_time(e1) / args.steps
    G = b.G
    value = G / (ms_per_step / 1e3)
    one_gps = one_by_one_s = None
    if not args.no_one_by_one:
        # one graph at a time through the single-graph path, same device-resident inputs
        views = []
        for i in range(G):
            d = b.desc[i]
            n, R = int(d["n"]), int(d["row_words"])
            a, o = int(d["row_offset"]), int(d["vertex_offset"])
            rows_v = b.rows[a:a + n * R].view(n, R)
            views.append((graph_bitset(rows_v), b.colour[o:o + n], int(d["k"]), b.vmask[o:o + n],
                          b.emask[a:a + n * R].view(n, R)))
        for gr, col, k, vm, em in views[:8]:
            kz.run(gr, col, k, vm, em)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        single = [kz.run(gr, col, k, vm, em) for gr, col, k, vm, em in views]
        torch.cuda.synchronize()
        one_by_one_s = time.perf_counter() - t0
        for i, r in enumerate(single):
            assert r["rounds"] == res[i]["rounds"] and r["surviving_edges"] == res[i]["surviving_edges"], i
        one_gps = G / one_by_one_s
    # algorithmic work: full-segment edge-test ops over the exact worklists
    ops = 0.0
    for i, (rows, colour, k) in enumerate(graphs):
        sizes = np.bincount(colour, minlength=k).astype(np.int64)
        words = (sizes + 63) // 64
        segoff = np.concatenate([[0], np.cumsum(words)])
        R = int(words.sum())
        pc = np.bitwise_count(rows).astype(np.int64)
        seg = np.add.reduceat(pc, segoff[:-1], axis=1) if R else np.zeros((rows.shape[0], k), np.int64)
        seg[:, words == 0] = 0
        cls_rows = np.add.reduceat(seg, np.concatenate([[0], np.cumsum(sizes)[:-1]]), axis=0)
        cls_rows[sizes == 0, :] = 0
        per_edge = 4 * (R - words[:, None] - words[None, :])
        m_g = max(int(res[i]["input_edges"]), 1)
        ops += float((np.triu(cls_rows, 1) * per_edge).sum()) * res[i]["edge_tests"] / m_g
    achieved = ops / (kernel_ms / 1e3) / 1e12
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import kernelize_bitset
        t0, done = time.perf_counter(), 0
        for rows, colour, k in graphs:
            kernelize_bitset(rows, colour, k)
            done += 1
            if time.perf_counter() - t0 > 15:
                break
        secs = time.perf_counter() - t0
        cpu = {"value": done / secs, "unit": "graphs/s", "cores": 1, "kind": "oracle",
               "sample": "the first %d graphs of the batch, one oracle fixpoint each (%.1f s)" % (done, secs)}
    out = {
        "metric": "batched graphs/s", "value": value, "unit": "graphs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "c4: " + WORKLOADS["c4"], "graphs": G, "vertices": int(b.desc["n"].sum()),
                   "edges": int(res["input_edges"].sum()), "max_rounds": int(res["rounds"].max()),
                   "mean_rounds": float(res["rounds"].mean()), "planted": None, "seed": args.seed,
                   "batch_config": tuned, "parallelism": "single GPU"},
        "one_by_one": None if one_gps is None else {
            "value": one_gps, "unit": "graphs/s", "seconds": one_by_one_s,
            "what": "kz_kernelize per graph on the same device-resident inputs"},
        "batched_over_one_by_one": None if one_gps is None else value / one_gps,
        "graph_capture_ms": round(capture_ms, 3),
        "roofline": {"kernel": "k_batch", "bound": "alu", "achieved": round(achieved, 3),
                     "peak": round(VALU_PEAK_TOPS, 2), "unit": "TFLOP/s", "frac": round(achieved / VALU_PEAK_TOPS, 4),
                     "traffic": traffic_from_profile("c4"),
                     "ops": "32-bit integer VALU ops (AND, OR) of the full-segment edge test, all graphs",
                     "avg_launch_ms": round(kernel_ms, 4), "alg_ops_per_launch": ops,
                     "valu_issue_frac": profile_value("c4", "valu_issue_frac"), "model_note": ALU_MODEL_NOTE},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """Config 5: continuous-batching server, closed-loop saturation and two
    Poisson open-loop rates, p50/p99 latency from arrival to completion."""
    import torch

    from paper_2212_00574_amd import inputs
    from paper_2212_00574_amd.binding import Kernelizer, Server, kz_gen_bitset
    N = args.requests
    specs = inputs.config5_specs(args.seed, requests=N)
    dev = torch.device("cuda", 0)
    kz = Kernelizer(0)
    bufs = []
    for sp in specs:
        n, R = int(sp.n), int(((sp.sizes + 63) // 64).sum())
        bufs.append({"n": n, "R": R, "k": int(sp.k),
                     "rows": torch.empty(n * R, dtype=torch.int64, device=dev),
                     "colour": torch.empty(n, dtype=torch.int32, device=dev),
                     "vmask": torch.empty(n, dtype=torch.uint8, device=dev),
                     "emask": torch.empty(n * R, dtype=torch.int64, device=dev)})
    srv = Server(kz, arena_bytes=8 << 30, max_slots=512)
    sid = srv.stream.cuda_stream
    gen = [False] * N

    def submit(i):
        b, sp = bufs[i], specs[i]
        if not gen[i]:   # materialise the request's rows on the server's stream
            kz_gen_bitset(kz.ctx, sp.sizes, sp.p, args.seed, i, None, b["rows"].data_ptr(), b["R"],
                          b["colour"].data_ptr(), sid)
            gen[i] = True
        return srv.submit(b["rows"], b["colour"], b["k"], b["vmask"], b["emask"])

    def run(arrivals):
        """Admits request i at arrivals[i] (seconds; None = as fast as admitted);
        returns (results, latency seconds, elapsed seconds)."""
        for i in range(N):
            gen[i] = False
        res, lat = [None] * N, np.zeros(N)
        fifo, backlog = [], []
        nxt, done, head = 0, 0, 0
        t0 = time.perf_counter()
        while done < N:
            now = time.perf_counter() - t0
            while nxt < N and (arrivals is None or arrivals[nxt] <= now):
                backlog.append(nxt)
                nxt += 1
            while backlog:
                t = submit(backlog[0])
                if t is None:
                    break
                fifo.append((t, backlog.pop(0)))
            srv.progress()
            # launches complete in admission order: poll from the oldest
            while head < len(fifo):
                t, i = fifo[head]
                r = srv.poll(t)
                if r is None:
                    break
                res[i] = r
                lat[i] = time.perf_counter() - t0 - (arrivals[i] if arrivals is not None else 0.0)
                head += 1
                done += 1
            if time.perf_counter() - t0 > 300:
                raise RuntimeError("serving run did not finish")
        return res, lat, time.perf_counter() - t0

    warm = N
    N = min(32, warm)
    run(None)                              # warm-up on the first requests
    N = warm
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(srv.stream)
    res, _, closed_s = run(None)
    e1.record(srv.stream)
    torch.cuda.synchronize()
    gpu_ms = e0.elapsed_time(e1)
    st = np.array([r["status"] for r in res])
    assert np.all(st == 0), np.unique(st)
    S = N / closed_s
    base_arr = np.array([sp.arrival_s for sp in specs])   # offered rate 1000/s in the specs
    phases = {}
    for frac in (0.5, 0.8):
        rate = frac * S
        arr = base_arr * (1000.0 / rate)
        r2, lat, el = run(arr)
        for i in range(N):
            assert r2[i]["edge_tests"] == res[i]["edge_tests"] and r2[i]["rounds"] == res[i]["rounds"], i
        phases["%.1fS" % frac] = {"offered_rps": rate, "achieved_rps": N / el, "p50_ms": float(np.percentile(lat, 50) * 1e3),
                                  "p99_ms": float(np.percentile(lat, 99) * 1e3), "max_ms": float(lat.max() * 1e3)}
        print("phase %.1fS: %s" % (frac, phases["%.1fS" % frac]), file=sys.stderr, flush=True)
    tests = np.array([r["edge_tests"] for r in res], dtype=np.float64)
    # full-segment ops: with near-equal classes every segment has R/k words
    # (to within one), so an edge test costs 4 R (k - 2) / k 32-bit ops
    ops = float(sum(tests[i] * 4.0 * bufs[i]["R"] * (bufs[i]["k"] - 2) / bufs[i]["k"] for i in range(N)))
    achieved = ops / (gpu_ms / 1e3) / 1e12
    # parity spot-check: the three smallest requests against the oracle
    from oracle import kernelize_bitset
    for i in sorted(range(N), key=lambda j: bufs[j]["n"] * bufs[j]["R"])[:3]:
        g = inputs.make_graph(specs[i].sizes, specs[i].p, seed=args.seed, gid=i, shuffle=False)
        rows, col, lay = g.bitset()
        ref = kernelize_bitset(rows, col, specs[i].k)
        assert ref["edge_tests"] == res[i]["edge_tests"] and ref["surv_edges"] == res[i]["surviving_edges"], i
        assert np.array_equal(bufs[i]["vmask"].cpu().numpy(), ref["vmask"]), i
    cpu = None
    if not args.no_cpu_baseline:
        t_or, done_n, tests_n = 0.0, 0, 0
        for i in sorted(range(N), key=lambda j: bufs[j]["n"]):
            g = inputs.make_graph(specs[i].sizes, specs[i].p, seed=args.seed, gid=i, shuffle=False)
            rows, col, lay = g.bitset()
            t0 = time.perf_counter()
            ref = kernelize_bitset(rows, col, specs[i].k)
            t_or += time.perf_counter() - t0
            done_n += 1
            tests_n += ref["edge_tests"]
            if t_or > 15:
                break
        cpu = {"value": tests_n / t_or, "unit": "edge tests/s", "cores": 1, "kind": "oracle",
               "sample": "the %d smallest of the %d requests, one oracle fixpoint each (%.1f s); the mix would take "
                         "%.0f s at this rate" % (done_n, N, t_or, tests.sum() / (tests_n / t_or))}
    out = {
        "metric": "served requests/s (closed loop)", "value": S, "unit": "requests/s", "n_gpus": 1,
        "steps": N, "warmup": 32, "ms_per_step": closed_s * 1e3 / N, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "c5: " + WORKLOADS["c5"], "requests": N, "seed": args.seed,
                   "edge_tests": float(tests.sum()), "max_rounds": int(max(r["rounds"] for r in res)),
                   "batch_config": None, "parallelism": "single GPU"},
        "latency": phases,
        "edge_tests_per_s": float(tests.sum()) / closed_s,
        "roofline": {"kernel": "k_batch (batch lane) and k_edge (single-graph lane), whole closed loop",
                     "bound": "alu", "achieved": round(achieved, 3),
                     "peak": round(VALU_PEAK_TOPS, 2), "unit": "TFLOP/s", "frac": round(achieved / VALU_PEAK_TOPS, 4),
                     "traffic": None, "ops": "32-bit VALU ops of the full-segment edge test over the exact worklists",
                     "gpu_stream_ms": round(gpu_ms, 3)},
        "cpu_baseline": cpu,
    }
    srv.close()
    print(json.dumps(out), flush=True)


def copy_calibration(mib):
    """Device-to-device copies of a known size, for scaling memory counters."""
    import torch
    n = mib * (1 << 20)
    a = torch.ones(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "copies": 5}), flush=True)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(a graph would shard by class columns, one block of classes per GPU).", file=sys.stderr)
        sys.exit(2)
    if args.workload == "c4":
        bench_batch(args)
        return
    if args.workload == "c5":
        bench_serve(args)
        return
    import torch

    from paper_2212_00574_amd.binding import KERNELS, Kernelizer

    dev = torch.device("cuda", 0)
    w = make_workload(args.workload, args.seed)
    print("workload %s ready" % args.workload, file=sys.stderr, flush=True)
    kz = Kernelizer(0)
    mfma = args.edge_path == "mfma"
    if mfma:
        if w["fmt"] == "csr":
            raise SystemExit("the MFMA edge path applies to dense and bit-row input")
        from paper_2212_00574_amd.binding import KZ_EDGE_MFMA_I8
        kz.set_edge_path(KZ_EDGE_MFMA_I8)
    # the input's copy to the device, timed on its own (the timed steps start
    # with the input resident; the library takes device buffers only)
    host_in = [w["colour"]] + ([w["adj"]] if w["fmt"] == "dense" else
                               [w["rp"], w["ci"]] if w["fmt"] == "csr" else [w["rows"]])
    h2d_bytes = int(sum(a.nbytes for a in host_in))
    e_h0, e_h1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    pinned = [torch.from_numpy(np.ascontiguousarray(a).view(np.uint8).reshape(-1)).pin_memory() for a in host_in]
    dev_copy = [torch.empty(t.shape, dtype=torch.uint8, device=dev) for t in pinned]
    for d, t in zip(dev_copy, pinned):   # first use of the copy path, untimed
        d.copy_(t, non_blocking=True)
    torch.cuda.synchronize()
    e_h0.record()
    for d, t in zip(dev_copy, pinned):
        d.copy_(t, non_blocking=True)
    e_h1.record()
    torch.cuda.synchronize()
    h2d_ms = e_h0.elapsed_time(e_h1)
    del pinned, dev_copy
    colour = torch.from_numpy(w["colour"]).to(dev)
    k = w["k"]
    if w["fmt"] == "dense":
        from paper_2212_00574_amd.binding import graph_dense
        x = torch.from_numpy(w["adj"]).to(dev)
        graph = graph_dense(x)
        n = x.shape[0]
        vmask = torch.empty(n, dtype=torch.uint8, device=dev)
        emask = torch.empty((n, n), dtype=torch.uint8, device=dev)
    elif w["fmt"] == "csr":
        from paper_2212_00574_amd.binding import graph_csr
        rp_t = torch.from_numpy(w["rp"]).to(dev)
        x = torch.from_numpy(w["ci"]).to(dev)
        graph = graph_csr(rp_t, x)
        n = rp_t.shape[0] - 1
        vmask = torch.empty(n, dtype=torch.uint8, device=dev)
        emask = torch.empty(x.shape[0], dtype=torch.uint8, device=dev)
    else:
        from paper_2212_00574_amd.binding import graph_bitset
        x = torch.from_numpy(w["rows"].view(np.int64)).to(dev)
        graph = graph_bitset(x)
        n = x.shape[0]
        vmask = torch.empty(n, dtype=torch.uint8, device=dev)
        emask = torch.empty_like(x)
    torch.cuda.synchronize()

    def step():
        return kz.run(graph, colour, k, vmask, emask)

    for _ in range(args.warmup):
        res = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = res["edge_tests"] / (ms_per_step / 1e3)
    # 20 steps timed one by one with HIP events on the stream: median and min
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(20)]
    for e0, e1 in ev:
        e0.record()
        step()
        e1.record()
    torch.cuda.synchronize()
    per_step = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
    print("timed %d steps: %.4f ms/step" % (args.steps, ms_per_step), file=sys.stderr, flush=True)

    # per-kernel times with HIP events on the launch stream (same workload, same launches)
    psteps = args.profile_steps or args.steps
    kz.profile(True)
    for _ in range(psteps):
        step()
    torch.cuda.synchronize()
    times = kz.kernel_times()
    kz.profile(False)
    edge_ms, edge_launches = times["edge"]
    edge_avg_ms = edge_ms / max(edge_launches, 1)
    passes = res["passes"]

    traffic = traffic_from_profile(args.workload)
    launches = max(edge_launches / psteps, 1)
    scale = res["edge_tests"] / max(res["input_edges"], 1)
    if w["fmt"] == "csr":
        # the sparse edge pass streams row entries: HBM-bound
        op_bytes, m_check = csr_operand_bytes(w)
        bytes_per_launch = op_bytes * scale / launches
        achieved = bytes_per_launch / (edge_avg_ms / 1e3) / 1e9
        roofline = {"kernel": "k_csr_edge", "bound": "hbm", "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                    "traffic": traffic, "alg_bytes_per_launch": bytes_per_launch,
                    "bytes": "4 (deg u + deg v) per tested edge",
                    "avg_launch_ms": round(edge_avg_ms, 5), "launches_per_step": edge_launches / psteps,
                    "traffic_GBps": None if traffic is None else round(traffic / (edge_avg_ms / 1e3) / 1e9, 1),
                    "model_note": CSR_MODEL_NOTE}
    elif mfma:
        # int8 MFMA counts: every pair of two classes against every third
        # class, 2 ops per multiply-accumulate, over the first (full) pass;
        # later passes recount only tiles with a touched block
        _, _, m_check = edge_work(w)
        sizes = np.asarray(w["sizes"], np.float64)
        n_all = sizes.sum()
        full = 0.0
        for a in range(len(sizes)):
            for b in range(a + 1, len(sizes)):
                full += 2.0 * sizes[a] * sizes[b] * (n_all - sizes[a] - sizes[b])
        ops_per_launch = full * (1.0 if res["passes"] == 1 else 1.0 / launches)
        achieved = ops_per_launch / (edge_avg_ms / 1e3) / 1e12
        roofline = {"kernel": "k_mfma_count + k_edge epilogue", "bound": "mfma", "achieved": round(achieved, 2),
                    "peak": I8_PEAK_TOPS, "unit": "TFLOP/s", "frac": round(achieved / I8_PEAK_TOPS, 4),
                    "traffic": None, "ops": "int8 MFMA ops (2 per multiply-accumulate) of the full-pass count",
                    "alg_ops_per_launch": ops_per_launch, "avg_launch_ms": round(edge_avg_ms, 5),
                    "launches_per_step": edge_launches / psteps}
    else:
        op_bytes, ops, m_check = edge_work(w)
        # exact-worklist work over all passes: pass 1 tests every edge; later
        # passes fewer (scaled by the tested-edge ratio)
        ops_per_launch = ops * scale / launches
        bytes_per_launch = op_bytes * scale / launches
        achieved = ops_per_launch / (edge_avg_ms / 1e3) / 1e12
        stream_gbps = bytes_per_launch / (edge_avg_ms / 1e3) / 1e9
        roofline = {
            "kernel": "k_edge",
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": round(VALU_PEAK_TOPS, 2),
            "unit": "TFLOP/s",
            "frac": round(achieved / VALU_PEAK_TOPS, 4),
            "traffic": traffic,
            "ops": "32-bit integer VALU ops (AND, OR) of the full-segment edge test",
            "alg_ops_per_launch": ops_per_launch,
            "avg_launch_ms": round(edge_avg_ms, 5),
            "launches_per_step": edge_launches / psteps,
            "operand_stream_GBps": round(stream_gbps, 1),
            "operand_stream_frac_of_hbm": round(stream_gbps / HBM_PEAK_GBPS, 3),
            "valu_issue_frac": profile_value(args.workload, "valu_issue_frac"),
            "model_note": ALU_MODEL_NOTE,
        }

    cpu = None
    check = None
    if not args.no_cpu_baseline and args.workload == "c3a":
        # the whole graph would keep the oracle busy for minutes: time it on a
        # smaller instance of the same recipe instead (k=20, p=0.3)
        from paper_2212_00574_amd import inputs
        gs = inputs.make_graph([200] * 20, 0.3, seed=args.seed, gid=1, shuffle=False)
        rows_s, col_s, _ = gs.bitset()
        sample = dict(fmt="bitset", rows=rows_s, colour=col_s, k=20)
        ores, _, secs, load_s = cpu_baseline(sample)
        cpu = {"value": ores["edge_tests"] / secs, "unit": "edge tests/s", "cores": 1, "kind": "oracle",
               "sample": "a smaller instance of the recipe (k=20 x 200, p=0.3), one oracle fixpoint "
                         "(%d edge tests, %.1f s; ingest %.1f s excluded)" % (ores["edge_tests"], secs, load_s)}
    elif not args.no_cpu_baseline:
        ores, (ovm, oem), secs, load_s = cpu_baseline(w)
        cpu = {"value": ores["edge_tests"] / secs, "unit": "edge tests/s", "cores": 1, "kind": "oracle",
               "sample": "the whole %s graph, one oracle fixpoint (%d edge tests, %.1f s; ingest %.1f s excluded)"
                         % (args.workload, ores["edge_tests"], secs, load_s)}
        gvm = vmask.cpu().numpy()
        gem = emask.cpu().numpy()
        if w["fmt"] == "bitset":
            gem = gem.view(np.uint64)
        check = bool(np.array_equal(gvm, ovm) and np.array_equal(gem, oem)
                     and ores["rounds"] == res["rounds"] and ores["edge_tests"] == res["edge_tests"])

    out = {
        "metric": "edge tests/s to fixpoint",
        "value": value,
        "unit": "edge tests/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "%s: %s" % (args.workload, WORKLOADS[args.workload]), "n": int(n), "k": int(k),
                   "edge_path": args.edge_path,
                   "edges": int(res["input_edges"]), "rounds": res["rounds"], "passes": passes,
                   "surviving_vertices": res["surviving_vertices"], "surviving_edges": res["surviving_edges"],
                   "seed": args.seed, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernel_ms_per_step": {name: round(t[0] / psteps, 5) for name, t in times.items()},
        "step_ms_median": round(per_step[len(per_step) // 2], 5),
        "step_ms_min": round(per_step[0], 5),
        "input_edges_per_s": res["input_edges"] / (ms_per_step / 1e3),
        "h2d": {"bytes": h2d_bytes, "ms": round(h2d_ms, 4),
                "what": "the input's copy from pinned host memory, outside the timed steps"},
        "oracle_equal": check,
    }
    assert m_check == res["input_edges"], (m_check, res["input_edges"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
