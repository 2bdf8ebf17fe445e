"""Benchmark: colour-index kernelization to the fixpoint on one MI355X.

Default run (no --workload): the headline line on the largest single-graph
workload, config 3a (k = 20 colour classes x 1000 vertices, inter-class edge
probability 0.3, class-major uint64 bit rows, 5.7e7 edges), with two
sub-objects in the same JSON line:

* ``batch`` -- config 4: 4096 graphs in one persistent launch under a
  captured hipGraph (batched graphs/s) against one-graph-at-a-time calls of
  the single-graph path on the same device-resident inputs;
* ``serve`` -- config 5: the 50,000-request stream through the server:
  closed-loop requests/s S, then Poisson arrivals at 0.5 S and 0.8 S with
  p50/p99 latency, and one-request-at-a-time calls on the same inputs.

A step of the headline is one full kz_kernelize call (validation, every pass
to the fixpoint, outputs) on inputs already resident in device memory;
``value`` is edge tests per second, counting the edge tests of the exact
worklists (every edge in the first pass; in pass r+1 the edges with an
endpoint that lost an edge in round r).  --workload c1 | c2 | c3a | c3b |
c4 | c5 runs one workload alone (used for the rocprofv3 summaries).

Inputs are seeded and synthetic (the generator of paper_2212_00574_amd/
inputs.py; kz_gen_bitset materialises the same graphs on the device).  The
CPU oracle runs only in the cpu_baseline leg, in a child process pinned to
one core.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import subprocess
import sys
import time

import numpy as np

# The serving workload runs the session lane, six single-graph workers and
# the caller's stream at once, after the other workloads have made streams
# of their own: give each stream a hardware queue of its own (HIP reads this
# when it starts, before any GPU call; streams beyond it share queues, and a
# stream that shares the session launch's queue waits for the launch).
os.environ.setdefault("GPU_MAX_HW_QUEUES", "16")

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0           # MI355X HBM3E, published
I8_PEAK_TOPS = 5000.0            # MI355X dense int8 MFMA, published (no sparsity)
# 32-bit integer VALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one wave64
# instruction per SIMD every 4 clocks); bitwise ops have no packed form.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
OPS_PER_WORD = 4                 # a 64-bit word tested: AND of two 32-bit halves, then OR/compare of both

WORKLOADS = {
    "c1": "k=4 classes x 25 vertices (n=100), p=0.5, dense uint8 input",
    "c2": "k=10 classes x 300 vertices (n=3000), p=0.6, planted 10-clique, uint64 bit rows",
    "c3a": "k=20 classes x 1000 vertices (n=20000), p=0.3, uint64 bit rows",
    "c3b": "k=30 multinomial classes, n=100000, 2.5M uniform inter-class edges (avg degree 50), CSR",
    "c4": "4096 graphs, k~U{4..16}, class sizes~U{8..128}, p~U[0.2,0.8], 10% planted k-clique, uint64 bit rows",
    "c5": "served requests: n log-uniform [200,20000], k~U{5..30} near-equal classes, p~U[0.1,0.9], Poisson "
          "arrivals, uint64 bit rows materialised on the device at arrival",
    "dom": "dominance reductions (section 4.3), vertex and edge mode, on the thesis's ten evaluation sizes "
           "n = 100, 300, ..., 1900 with n(n-5)/2 edges (path plus skewed edges), plain bit rows",
    "clique": "k-clique search on the 4096 batching graphs (config 4), on each input graph and on its kernel",
    "colours": "the 4096 batching graphs (config 4) with clique size k-2 below their k colour classes "
               "(thresholds k-3 and k-4), batched runtime",
    "colouring": "upstream legal colouring (Jones-Plassmann) of uncoloured G(n, p) graphs: n = 3000 at p = 0.3 "
                 "and n = 20000 at p = 0.05, seeded uint64 priorities",
    "struction": "struction (section 4.1) of a random graph of 1000 vertices at p = 0.1 around vertex 0 "
                 "(G' about 40 000 nodes), plain bit rows",
}
SERVE_SPLIT_N = 1024       # c5 lane split (vertices): below the library's 2048, as the session lane's
                           # largest jobs set the small requests' tail
SERVE_IDLE_US = 20000
SERVE_RESIDENT_GIB = 8.0
SERVE_WORKERS = 6          # c5: single-graph lane workers
DOM_SIZES = list(range(100, 2000, 200))
DOM_CPU_EDGE_SIZES = (100, 300, 500, 700, 900)   # edge-mode oracle sample: about 14 s on one core


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="headline", choices=["headline"] + sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-one-by-one", action="store_true",
                    help="c4/c5: skip the one-graph-at-a-time comparison (for counter runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=None,
                    help="steps of the per-kernel event-timed loop (default: --steps)")
    ap.add_argument("--edge-path", default="bitset", choices=("bitset", "mfma"),
                    help="edge test of the single-graph path: witness search on bit rows, or int8 MFMA counts")
    ap.add_argument("--requests", type=int, default=50000, help="c5: requests of the stream (a prefix)")
    ap.add_argument("--split-n", type=int, default=SERVE_SPLIT_N,
                    help="c5: requests of at least this many vertices take the single-graph lane")
    ap.add_argument("--idle-us", type=int, default=SERVE_IDLE_US, help="c5: a session launch ends after this idle time")
    ap.add_argument("--session-cus", type=int, default=0, help="c5: compute units of a session launch (0: 3/16)")
    ap.add_argument("--lease-us", type=int, default=0, help="c5: session workgroup lease (0: the server's 10 ms)")
    ap.add_argument("--workers", type=int, default=SERVE_WORKERS,
                    help="c5: single-graph lane workers (requests of that lane in flight at once)")
    ap.add_argument("--resident-gib", type=float, default=SERVE_RESIDENT_GIB,
                    help="c5: admission limit on the admitted requests' rows, colours and masks")
    ap.add_argument("--copy-calibration", type=int, default=None, metavar="MIB",
                    help="only run device-to-device copies of MIB MiB (memory-counter calibration)")
    return ap.parse_args(argv)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


# --------------------------------------------------------------- counters
# The kernel whose launches set each workload's roofline, and the sources it
# is built from (a committed counter summary is used only while they match).
PROFILED = {
    "c1": ("k_edge", ("kz_kernels.hip", "kz_internal.h")),
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


def source_hash(workload="c3a"):
    """Hash of the code (comments and layout ignored) the workload's roofline
    kernel is built from."""
    h = hashlib.sha256()
    for f in PROFILED.get(workload, PROFILED["c3a"])[1]:
        h.update(_code_only(open(os.path.join(ROOT, "paper_2212_00574_amd", "csrc", f)).read()).encode())
    return h.hexdigest()[:16]


def profile_value(workload, key, kernel=None):
    """A figure ("- key: value") of the committed counter summary
    profiles/<kernel>_<workload>.md (default: the workload's roofline
    kernel); None when absent or when the kernel's sources changed since the
    counters were taken ("- source_sha: S")."""
    kernel = kernel or PROFILED.get(workload, PROFILED["c3a"])[0]
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


# --------------------------------------------------------------- host facts
def host_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count(), "allowed_cpus": len(os.sched_getaffinity(0))}


def digest(vmask, emask, r):
    """SHA-256 of vmask || emask (uint64 LE) || int64 LE [rounds, surviving
    vertices, surviving edges, edge tests]: the fingerprint the committed
    full-size fixtures hold (tests/golden/)."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(vmask, np.uint8).tobytes())
    h.update(np.ascontiguousarray(emask).view(np.uint64).astype("<u8", copy=False).tobytes())
    h.update(np.array([r["rounds"], r["surviving_vertices"], r["surviving_edges"], r["edge_tests"]],
                      "<i8").tobytes())
    return h.digest()


def golden(name):
    path = os.path.join(ROOT, "tests", "golden", name)
    return json.load(open(path)) if os.path.exists(path) else None


# --------------------------------------------------------------- CPU baseline
def _cpu_child(workload, seed):
    """Runs in a child process pinned to one core (no GPU): the oracle on the
    workload, plus the witness-search word count of the bit-row input."""
    from oracle import FMT_CSR, FMT_DENSE, OracleGraph, fixpoint_rows, witness_words
    from paper_2212_00574_amd import inputs
    out = {}
    t0 = time.perf_counter()
    if workload == "c1":
        g = inputs.config1(seed)
        adj, colour = g.dense()
        t1 = time.perf_counter()
        og = OracleGraph(FMT_DENSE, len(colour), 4, colour, adj=adj)
        t2 = time.perf_counter()
        r = og.fixpoint()
        out.update(oracle="O1", edge_tests=r["edge_tests"], rounds=r["rounds"])
    elif workload == "c3b":
        sg = inputs.config3b(seed)
        t1 = time.perf_counter()
        og = OracleGraph(FMT_CSR, sg.n, sg.k, sg.colour, row_ptr=sg.row_ptr, col_idx=sg.col_idx)
        t2 = time.perf_counter()
        r = og.fixpoint()
        out.update(oracle="O1", edge_tests=r["edge_tests"], rounds=r["rounds"])
    else:
        g = inputs.config2(seed) if workload == "c2" else inputs.config3a(seed)
        rows, colour, lay = g.bitset()
        t1 = time.perf_counter()
        t2 = t1
        r = fixpoint_rows(rows, colour, g.k)
        out.update(oracle="O3", edge_tests=r["edge_tests"], rounds=r["rounds"])
    t3 = time.perf_counter()
    out.update(gen_s=t1 - t0, ingest_s=t2 - t1, fixpoint_s=t3 - t2)
    if workload in ("c2", "c3a"):
        t4 = time.perf_counter()
        out["witness"] = witness_words(rows, colour, g.k)
        out["witness_s"] = time.perf_counter() - t4
    print(json.dumps(out), flush=True)


def start_cpu_child(workload, seed):
    """Starts the oracle child on the last allowed core (before any GPU use)."""
    cpus = sorted(os.sched_getaffinity(0))
    core = cpus[-1]
    code = ("import os, sys; os.sched_setaffinity(0, {%d}); sys.path.insert(0, %r); import bench; "
            "bench._cpu_child(%r, %d)" % (core, ROOT, workload, seed))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    p = subprocess.Popen([sys.executable, "-c", code], stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True,
                         env=env)
    return p, core


def finish_cpu_child(proc, core, workload):
    out, err = proc.communicate(timeout=900)
    if proc.returncode != 0:
        say("cpu baseline child failed:", err[-2000:])
        return None, None
    d = json.loads(out.strip().splitlines()[-1])
    secs = d["fixpoint_s"]
    what = {"O1": "the oracle's synchronous rounds on adjacency lists (O1)",
            "O3": "the oracle's synchronous rounds on bit rows (O3, the same result as O1)"}[d["oracle"]]
    cpu = {"value": d["edge_tests"] / secs, "unit": "edge tests/s", "cores": 1, "kind": "oracle",
           "sample": "the whole %s graph: %s to the fixpoint, %d edge tests in %.2f s on one core (pinned to "
                     "cpu %d; generation %.1f s and ingest %.1f s excluded)"
                     % (workload, what, d["edge_tests"], secs, core, d["gen_s"], d["ingest_s"]),
           "host": host_info()}
    return cpu, d


def _dom_cpu_child(seed):
    """Child process pinned to one core: the dominance oracle's times (vertex
    mode on every evaluation graph, edge mode on DOM_CPU_EDGE_SIZES)."""
    from oracle import dom_edge, dom_vertex
    from paper_2212_00574_amd import inputs
    out = {"vertex": {}, "edge": {}}
    for n in DOM_SIZES:
        adj = inputs.dominance_graph(n, seed)
        t0 = time.perf_counter()
        dom_vertex(adj)
        out["vertex"][n] = time.perf_counter() - t0
        if n in DOM_CPU_EDGE_SIZES:
            t0 = time.perf_counter()
            dom_edge(adj)
            out["edge"][n] = time.perf_counter() - t0
    print(json.dumps(out), flush=True)


def start_dom_cpu_child(seed):
    cpus = sorted(os.sched_getaffinity(0))
    core = cpus[-2] if len(cpus) > 1 else cpus[-1]
    code = ("import os, sys; os.sched_setaffinity(0, {%d}); sys.path.insert(0, %r); import bench; "
            "bench._dom_cpu_child(%d)" % (core, ROOT, seed))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    p = subprocess.Popen([sys.executable, "-c", code], stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True,
                         env=env)
    return p, core


# --------------------------------------------------------------- single graph
def class_pair_edges(rows_host, sizes):
    """Edges between every pair of classes of a bit-row graph (host side)."""
    sizes = np.asarray(sizes, np.int64)
    k = len(sizes)
    words = (sizes + 63) // 64
    segoff = np.concatenate([[0], np.cumsum(words)])
    pc = np.bitwise_count(rows_host.view(np.uint64)).astype(np.int64)
    seg = np.zeros((rows_host.shape[0], k), np.int64)
    for c in range(k):
        if words[c]:
            seg[:, c] = pc[:, segoff[c]:segoff[c + 1]].sum(axis=1)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    cnt = np.zeros((k, k), np.int64)
    for a in range(k):
        cnt[a] = seg[offs[a]:offs[a + 1]].sum(axis=0)
    return cnt


def full_segment_work(cnt, sizes):
    """Full-segment model of one sweep: operand bytes 2 (n - s_cu - s_cv) / 8
    per edge (both rows streamed) and 4 ops per word of every third class."""
    sizes = np.asarray(sizes, np.int64)
    n = int(sizes.sum())
    words = (sizes + 63) // 64
    R = int(words.sum())
    k = len(sizes)
    op_bytes = ops = 0.0
    for a in range(k):
        for b in range(a + 1, k):
            m_ab = float(cnt[a, b])
            op_bytes += m_ab * 2 * (n - sizes[a] - sizes[b]) / 8
            ops += m_ab * OPS_PER_WORD * (R - words[a] - words[b])
    return op_bytes, ops, int(np.triu(cnt, 1).sum())


def make_single(name, seed, kz, dev):
    """(graph descriptor, colour, k, vmask, emask, sizes, host rows or None)
    with the input resident in device memory."""
    import torch

    from paper_2212_00574_amd import inputs
    from paper_2212_00574_amd.binding import graph_bitset, graph_csr, graph_dense, kz_gen_bitset
    if name == "c1":
        g = inputs.config1(seed)
        adj, colour = g.dense()
        x = torch.from_numpy(adj).to(dev)
        n = x.shape[0]
        return (graph_dense(x), torch.from_numpy(colour).to(dev), 4, torch.empty(n, dtype=torch.uint8, device=dev),
                torch.empty((n, n), dtype=torch.uint8, device=dev), g.sizes, None, [x])
    if name == "c3b":
        sg = inputs.config3b(seed)
        rp = torch.from_numpy(sg.row_ptr).to(dev)
        ci = torch.from_numpy(sg.col_idx).to(dev)
        n = sg.n
        return (graph_csr(rp, ci), torch.from_numpy(sg.colour).to(dev), sg.k,
                torch.empty(n, dtype=torch.uint8, device=dev), torch.empty(ci.shape[0], dtype=torch.uint8, device=dev),
                sg.sizes, None, [rp, ci])
    g = inputs.config2(seed) if name == "c2" else inputs.config3a(seed)
    lay = inputs.class_layout(g.sizes)
    rows = torch.empty((lay.n, lay.R), dtype=torch.int64, device=dev)
    colour = torch.empty(lay.n, dtype=torch.int32, device=dev)
    kz_gen_bitset(kz.ctx, g.sizes, g.p, seed, 0, g.planted, rows.data_ptr(), lay.R, colour.data_ptr(), None)
    torch.cuda.synchronize()
    return (graph_bitset(rows), colour, g.k, torch.empty(lay.n, dtype=torch.uint8, device=dev), torch.empty_like(rows),
            g.sizes, rows, [rows])


def run_single(args, name, cpu_proc=None):
    import torch

    from paper_2212_00574_amd.binding import KZ_EDGE_MFMA_I8, Kernelizer
    dev = torch.device("cuda", 0)
    kz = Kernelizer(0)
    mfma = args.edge_path == "mfma"
    if mfma:
        if name in ("c1", "c3b"):
            raise SystemExit("the MFMA edge path is measured on bit-row input")
        kz.set_edge_path(KZ_EDGE_MFMA_I8)
    graph, colour, k, vmask, emask, sizes, rows_dev, keep = make_single(name, args.seed, kz, dev)
    say("workload %s resident on the device" % name)
    # the input's copy from pinned host memory, timed on its own (never in value)
    nbytes = int(sum(t.numel() * t.element_size() for t in keep) + colour.numel() * 4)
    pinned = torch.empty(nbytes, dtype=torch.uint8).pin_memory()
    dcopy = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    dcopy.copy_(pinned, non_blocking=True)
    torch.cuda.synchronize()
    e_h0, e_h1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e_h0.record()
    dcopy.copy_(pinned, non_blocking=True)
    e_h1.record()
    torch.cuda.synchronize()
    h2d_ms = e_h0.elapsed_time(e_h1)
    del pinned, dcopy

    def step():
        return kz.run(graph, colour, k, vmask, emask)

    for _ in range(args.warmup):
        res = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / args.steps
    value = res["edge_tests"] / (ms_per_step / 1e3)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(20)]
    for e0, e1 in ev:
        e0.record()
        step()
        e1.record()
    torch.cuda.synchronize()
    per_step = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
    say("%s: %d steps, %.4f ms/step" % (name, args.steps, ms_per_step))

    # per-kernel times with HIP events on the launch stream (same launches)
    psteps = args.profile_steps or args.steps
    kz.profile(True)
    for _ in range(psteps):
        step()
    torch.cuda.synchronize()
    times = kz.kernel_times()
    kz.profile(False)
    edge_ms, edge_launches = times["edge"]
    edge_avg_ms = edge_ms / max(edge_launches, 1)
    launches = max(edge_launches / psteps, 1)
    scale = res["edge_tests"] / max(res["input_edges"], 1)   # exact-worklist tests over one full sweep

    # parity with the committed oracle fixture (the whole graph)
    check = None
    fx = golden("%s_seed%d.json" % (name, args.seed))
    if fx is not None and not mfma:
        d = digest(vmask.cpu().numpy(), emask.cpu().numpy(), res)
        check = d.hex() == fx["sha256"]

    cpu, child = (None, None)
    if cpu_proc is not None:
        cpu, child = finish_cpu_child(*cpu_proc, name)

    traffic = traffic_from_profile(name)
    if name == "c3b":
        from paper_2212_00574_amd import inputs
        sg = inputs.config3b(args.seed)
        deg = np.diff(sg.row_ptr).astype(np.int64)
        src = np.repeat(np.arange(len(deg)), deg)
        up = src < sg.col_idx
        op_bytes = float(4 * (deg[src[up]] + deg[sg.col_idx[up]]).sum())
        m_check = int(up.sum())
        bytes_per_launch = op_bytes * scale / launches
        achieved = bytes_per_launch / (edge_avg_ms / 1e3) / 1e9
        roofline = {"kernel": "k_csr_edge", "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                    "bytes": "4 (deg u + deg v) per tested edge", "alg_bytes_per_launch": bytes_per_launch,
                    "avg_launch_ms": round(edge_avg_ms, 5), "launches_per_step": edge_launches / psteps,
                    "note": "the two rows of an edge are re-read from L2 and the Infinity Cache, so this stream "
                            "can pass the HBM peak; traffic is the counter-measured HBM bytes per launch"}
    elif name == "c1":
        m_check = res["input_edges"]
        roofline = {"kernel": "k_edge", "bound": "launch latency", "achieved": None, "peak": None, "unit": None,
                    "frac": None, "traffic": None, "avg_launch_ms": round(edge_avg_ms, 5),
                    "note": "100 vertices: every kernel is one or two workgroups; the step is launch latency"}
    else:
        rows_host = rows_dev.cpu().numpy()
        cnt = class_pair_edges(rows_host, sizes)
        op_bytes, fs_ops, m_check = full_segment_work(cnt, sizes)
        if mfma:
            s = np.asarray(sizes, np.float64)
            n_all = s.sum()
            full = sum(2.0 * s[a] * s[b] * (n_all - s[a] - s[b]) for a in range(len(s)) for b in range(a + 1, len(s)))
            ops_per_launch = full * (1.0 if res["passes"] == 1 else 1.0 / launches)
            achieved = ops_per_launch / (edge_avg_ms / 1e3) / 1e12
            roofline = {"kernel": "k_mfma_count + k_edge_mf", "bound": "mfma", "achieved": round(achieved, 2),
                        "peak": I8_PEAK_TOPS, "unit": "TFLOP/s", "frac": round(achieved / I8_PEAK_TOPS, 4),
                        "traffic": None, "ops": "int8 MFMA ops (2 per multiply-accumulate) of the full count",
                        "alg_ops_per_launch": ops_per_launch, "avg_launch_ms": round(edge_avg_ms, 5),
                        "launches_per_step": edge_launches / psteps}
        else:
            wit = child["witness"] if child and "witness" in child else None
            need_ops = None if wit is None else OPS_PER_WORD * wit["words"] * scale / launches
            fs_per_launch = fs_ops * scale / launches
            achieved = None if need_ops is None else need_ops / (edge_avg_ms / 1e3) / 1e12
            fs_achieved = fs_per_launch / (edge_avg_ms / 1e3) / 1e12
            stream_gbps = op_bytes * scale / launches / (edge_avg_ms / 1e3) / 1e9
            roofline = {
                "kernel": "k_edge", "bound": "alu",
                "achieved": None if achieved is None else round(achieved, 3),
                "peak": round(VALU_PEAK_TOPS, 2), "unit": "TFLOP/s",
                "frac": None if achieved is None else round(achieved / VALU_PEAK_TOPS, 4),
                "traffic": traffic,
                "ops": "necessary 32-bit ops of a first-witness search: %d per 64-bit word read, over the words "
                       "up to the first common neighbour of every (edge, third class) pair (oracle-side count)"
                       % OPS_PER_WORD,
                "alg_ops_per_launch": need_ops, "witness": wit,
                "avg_launch_ms": round(edge_avg_ms, 5), "launches_per_step": edge_launches / psteps,
                "full_segment": {"ops_per_launch": fs_per_launch, "achieved": round(fs_achieved, 3),
                                 "frac": round(fs_achieved / VALU_PEAK_TOPS, 4),
                                 "note": "every word of every third class (the full-segment model); a search that "
                                         "stops at the first witness does less, so this can pass 1"},
                "operand_stream": {"GBps": round(stream_gbps, 1), "frac_of_hbm": round(stream_gbps / HBM_PEAK_GBPS, 3),
                                   "note": "both rows streamed per edge, 2 (n - s_u - s_v)/8 bytes: the bandwidth a "
                                           "sweep with no reuse would need; reuse-bound, not HBM-bound"},
                "valu_issue_frac": profile_value(name, "valu_issue_frac"),
            }
    assert m_check == res["input_edges"], (m_check, res["input_edges"])
    stream = None
    if name in ("c2", "c3a") and not mfma and res["passes"] == 1:
        # pass 1's streaming kernel: reads the rows and colours, writes the
        # state, the first- and second-word matrices and the vertex mask
        n_v, r_w = int(vmask.numel()), int(rows_dev.numel()) // max(int(vmask.numel()), 1)
        chunk = 4 if k <= 4 else ((k + 3) // 4 * 4 if k <= 32 else 32)
        kf = (k + chunk - 1) // chunk * chunk
        vbytes = 16.0 * n_v * r_w + 16.0 * n_v * kf + 5.0 * n_v
        v_ms = times["vertex"][0] / max(times["vertex"][1], 1)
        v_gbps = vbytes / (v_ms / 1e3) / 1e9
        stream = {"kernel": "k_vertex_first", "bound": "hbm", "achieved": round(v_gbps, 1), "peak": HBM_PEAK_GBPS,
                  "unit": "GB/s", "frac": round(v_gbps / HBM_PEAK_GBPS, 4), "alg_bytes_per_launch": vbytes,
                  "bytes": "rows read + state written (8 n R each), F and S written (8 n kF each), colours and mask",
                  "avg_launch_ms": round(v_ms, 5),
                  "traffic": profile_value(name, "hbm_bytes_per_launch", "k_vertex_first")}
    out = {
        "metric": "edge tests/s to fixpoint", "value": value, "unit": "edge tests/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "%s: %s" % (name, WORKLOADS[name]), "n": int(vmask.numel()), "k": int(k),
                   "edge_path": args.edge_path, "edges": int(res["input_edges"]), "rounds": res["rounds"],
                   "passes": res["passes"], "surviving_vertices": res["surviving_vertices"],
                   "surviving_edges": res["surviving_edges"], "seed": args.seed, "parallelism": "single GPU"},
        "roofline": roofline,
        "stream_kernel": stream,
        "cpu_baseline": cpu,
        "kernel_ms_per_step": {nm: round(t[0] / psteps, 5) for nm, t in times.items()},
        "step_ms_median": round(per_step[len(per_step) // 2], 5), "step_ms_min": round(per_step[0], 5),
        "input_edges_per_s": res["input_edges"] / (ms_per_step / 1e3),
        "h2d": {"bytes": nbytes, "ms": round(h2d_ms, 4),
                "what": "the input's size copied from pinned host memory, outside the timed steps"},
        "oracle_equal": check,
    }
    kz.close()
    return out


# --------------------------------------------------------------- batch (c4)
def run_batch(args):
    """Config 4: batched graphs/s against one-graph-at-a-time launches."""
    import torch

    from paper_2212_00574_amd import inputs
    from paper_2212_00574_amd.binding import Batch, BatchKernelizer, Kernelizer, graph_bitset, kz_gen_bitset
    dev = torch.device("cuda", 0)
    kz = Kernelizer(0)
    specs = inputs.config4_specs(args.seed)
    shapes = [(int(sp.sizes.sum()), int(((sp.sizes + 63) // 64).sum()), sp.k) for sp in specs]
    b = Batch.allocate(shapes, dev)
    planted = 0
    for i, sp in enumerate(specs):
        d = b.desc[i]
        a, o = int(d["row_offset"]), int(d["vertex_offset"])
        pl = inputs.config4_graph(sp, args.seed, i).planted
        planted += pl is not None
        kz_gen_bitset(kz.ctx, sp.sizes, sp.p, args.seed, i, pl, b.rows[a:].data_ptr(), int(d["row_words"]),
                      b.colour[o:].data_ptr(), None)
    torch.cuda.synchronize()
    say("c4: %d graphs resident" % b.G)
    bk = BatchKernelizer(kz)
    tuned = bk.autotune(b)
    bk.run(b)
    torch.cuda.synchronize()
    res = b.read_results()
    assert np.all(res["status"] == 0), np.unique(res["status"])
    # parity: every graph's fingerprint against the oracle's (committed fixture)
    check = None
    fx = golden("c4_seed%d.json" % args.seed)
    if fx is not None:
        vm_all, em_all = b.vmask.cpu().numpy(), b.emask.cpu().numpy()
        check = True
        for bk_ in fx["buckets"]:
            lo, hi = bk_["ids"]
            h = hashlib.sha256()
            for i in range(lo, hi + 1):
                d = b.desc[i]
                n, R = int(d["n"]), int(d["row_words"])
                a, o = int(d["row_offset"]), int(d["vertex_offset"])
                r = {key: int(res[i][key]) for key in ("rounds", "surviving_vertices", "surviving_edges",
                                                       "edge_tests")}
                h.update(digest(vm_all[o:o + n], em_all[a:a + n * R], r))
            check = check and h.hexdigest() == bk_["hash"]
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
    ms_per_step = (time.perf_counter() - t0) * 1e3 / args.steps
    kernel_ms = e0.elapsed_time(e1) / args.steps
    value = b.G / (ms_per_step / 1e3)
    one = None
    if not args.no_one_by_one:
        views = []
        for i in range(b.G):
            d = b.desc[i]
            n, R = int(d["n"]), int(d["row_words"])
            a, o = int(d["row_offset"]), int(d["vertex_offset"])
            views.append((graph_bitset(b.rows[a:a + n * R].view(n, R)), b.colour[o:o + n], int(d["k"]),
                          b.vmask[o:o + n], b.emask[a:a + n * R].view(n, R)))
        for gr, col, k, vm, em in views[:8]:
            kz.run(gr, col, k, vm, em)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        single = [kz.run(gr, col, k, vm, em) for gr, col, k, vm, em in views]
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        same = all(r["rounds"] == res[i]["rounds"] and r["edge_tests"] == res[i]["edge_tests"]
                   and r["surviving_edges"] == res[i]["surviving_edges"] for i, r in enumerate(single))
        one = {"value": b.G / secs, "unit": "graphs/s", "seconds": secs, "same_results": same,
               "what": "kz_kernelize per graph on the same device-resident inputs"}
    say("c4: %.3f ms/batch" % ms_per_step)
    kz.close()
    return {"metric": "batched graphs/s", "value": value, "unit": "graphs/s", "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms_per_step, "kernel_ms_per_step": kernel_ms,
            "config": {"workload": "c4: " + WORKLOADS["c4"], "graphs": b.G, "vertices": int(b.desc["n"].sum()),
                       "edges": int(res["input_edges"].sum()), "planted": planted,
                       "mean_rounds": float(res["rounds"].mean()), "max_rounds": int(res["rounds"].max()),
                       "batch_config": tuned, "seed": args.seed},
            "one_by_one": one, "batched_over_one_by_one": None if one is None else value / one["value"],
            "graph_capture_ms": round(capture_ms, 3),
            "roofline": {"kernel": "k_batch", "traffic": traffic_from_profile("c4"),
                         "valu_issue_frac": profile_value("c4", "valu_issue_frac"),
                         "note": "counter figures from the committed summary (null once the kernel changed)"},
            "oracle_equal": check}


# --------------------------------------------------------------- serving (c5)
class Stream5:
    """The served requests' device buffers: materialised on the server's
    stream when first admitted, released when the request completes."""

    def __init__(self, kz, srv, specs, seed):
        self.kz, self.srv, self.specs, self.seed = kz, srv, specs, seed
        self.live = {}

    def buffers(self, i):
        import torch

        from paper_2212_00574_amd import inputs
        from paper_2212_00574_amd.binding import kz_gen_bitset
        if i not in self.live:
            sp = self.specs[i]
            lay = inputs.class_layout(sp.sizes)
            dev = self.kz.device
            rows = torch.empty((lay.n, lay.R), dtype=torch.int64, device=dev)
            colour = torch.empty(lay.n, dtype=torch.int32, device=dev)
            kz_gen_bitset(self.kz.ctx, sp.sizes, sp.p, self.seed, i, None, rows.data_ptr(), lay.R,
                          colour.data_ptr(), self.srv.stream.cuda_stream)
            self.live[i] = (rows, colour, torch.empty(lay.n, dtype=torch.uint8, device=dev), torch.empty_like(rows))
        return self.live[i]


def run_serve(args):
    """Config 5: the request stream through the server (continuous batching):
    closed-loop requests/s S, then Poisson arrivals at 0.5 S and 0.8 S."""
    import torch

    from paper_2212_00574_amd import inputs
    from paper_2212_00574_amd.binding import Kernelizer, Server, graph_bitset
    N = args.requests
    specs = inputs.config5_specs(args.seed, requests=N)
    kz = Kernelizer(0)
    # inputs are generated and fenced on a stream of the server's own, not
    # on the legacy null stream
    srv = Server(kz, arena_bytes=16 << 30, max_slots=512, stream=torch.cuda.Stream(kz.device))
    resident = int(args.resident_gib * (1 << 30))
    srv.configure(split_n=args.split_n, idle_us=args.idle_us, resident_limit=resident,
                  session_cus=args.session_cus, lease_us=args.lease_us, workers=args.workers)
    fx = golden("c5_seed%d.json" % args.seed)
    check_ids = set(fx["buckets"][0]["ids"]) if fx is not None and N == 50000 else set()
    digests = {}

    def run(arrivals):
        st = Stream5(kz, srv, specs, args.seed)
        res, lat = [None] * N, np.zeros(N)
        waiting, tickets = [], {}
        nxt, done = 0, 0
        t0 = time.perf_counter()
        while done < N:
            now = time.perf_counter() - t0
            while nxt < N and (arrivals is None or arrivals[nxt] <= now):
                waiting.append(nxt)
                nxt += 1
            while waiting:
                i = waiting[0]
                rows, colour, vm, em = st.buffers(i)
                t = srv.submit(rows, colour, specs[i].k, vm, em)
                if t is None:
                    break
                tickets[t] = i
                waiting.pop(0)
            for t, r in srv.done(1024):
                i = tickets.pop(t)
                res[i] = r
                lat[i] = time.perf_counter() - t0 - (arrivals[i] if arrivals is not None else 0.0)
                if arrivals is None and i in check_ids:
                    # complete once reported done; no device-wide wait (it
                    # would also wait for the running session launch to end)
                    _, _, vm, em = st.live[i]
                    digests[i] = digest(vm.cpu().numpy(), em.cpu().numpy(), r)
                st.live.pop(i, None)
                done += 1
                if done % 5000 == 0:
                    say("c5: %d of %d requests done, %.1f s" % (done, N, time.perf_counter() - t0))
            if time.perf_counter() - t0 > 400:
                raise RuntimeError("serving run did not finish")
        return res, lat, time.perf_counter() - t0

    N_all = N
    N = min(64, N_all)
    say("c5: warm-up on %d requests (split_n %d, idle %d us, resident limit %.1f GiB, %d workers)"
        % (N, args.split_n, args.idle_us, args.resident_gib, args.workers))
    run(None)                                   # warm-up on the first requests
    N = N_all
    res, _, closed_s = run(None)
    st_ = np.array([r["status"] for r in res])
    assert np.all(st_ == 0), np.unique(st_)
    S = N / closed_s
    say("c5: closed loop %.0f requests/s" % S)
    check = None
    if check_ids:
        h = hashlib.sha256()
        for i in fx["buckets"][0]["ids"]:
            h.update(digests[i])
        check = h.hexdigest() == fx["buckets"][0]["hash"]
    base_arr = np.array([sp.arrival_s for sp in specs])   # offered rate 1000/s in the specs
    small = np.array([sp.n < args.split_n for sp in specs])   # the session lane's requests

    def pct(x):
        return {"requests": int(x.size), "p50_ms": float(np.percentile(x, 50) * 1e3),
                "p99_ms": float(np.percentile(x, 99) * 1e3), "max_ms": float(x.max() * 1e3)} if x.size else None

    phases = {}
    for frac in (0.5, 0.8):
        rate = frac * S
        r2, lat, el = run(base_arr * (1000.0 / rate))
        same = all(r2[i]["edge_tests"] == res[i]["edge_tests"] and r2[i]["rounds"] == res[i]["rounds"]
                   and r2[i]["surviving_edges"] == res[i]["surviving_edges"] for i in range(N))
        phases["%.1fS" % frac] = {"offered_rps": rate, "achieved_rps": N / el,
                                  "p50_ms": float(np.percentile(lat, 50) * 1e3),
                                  "p99_ms": float(np.percentile(lat, 99) * 1e3), "max_ms": float(lat.max() * 1e3),
                                  "by_lane": {"session (n < split_n)": pct(lat[small]),
                                              "single_graph (n >= split_n)": pct(lat[~small])},
                                  "same_results_as_closed_loop": same}
        say("c5 phase %.1fS: %s" % (frac, phases["%.1fS" % frac]))
    srv.close()
    one = None
    if not args.no_one_by_one:
        st = Stream5(kz, srv, specs, args.seed)
        srv.stream = torch.cuda.current_stream()
        t_total, same = 0.0, True
        for i in range(N):
            rows, colour, vm, em = st.buffers(i)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = kz.run(graph_bitset(rows), colour, specs[i].k, vm, em)
            t_total += time.perf_counter() - t0
            same = same and r["edge_tests"] == res[i]["edge_tests"] and r["rounds"] == res[i]["rounds"]
            st.live.pop(i)
        one = {"value": N / t_total, "unit": "requests/s", "seconds": t_total, "same_results": same,
               "what": "kz_kernelize per request on the same device-resident inputs (materialisation excluded)"}
    tests = np.array([r["edge_tests"] for r in res], dtype=np.float64)
    kz.close()
    return {"metric": "served requests/s (closed loop)", "value": S, "unit": "requests/s", "requests": N,
            "ms_per_request": closed_s * 1e3 / N,
            "config": {"workload": "c5: " + WORKLOADS["c5"], "requests": N, "seed": args.seed,
                       "split_n": args.split_n, "idle_us": args.idle_us, "resident_limit_bytes": resident,
                       "session_cus": args.session_cus or "3/16 of the device", "lease_us": args.lease_us or 10000,
                       "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES"),
                       "workers": args.workers,
                       "max_slots": 512,
                       "edge_tests": float(tests.sum()), "max_rounds": int(max(r["rounds"] for r in res))},
            "latency": phases, "edge_tests_per_s": float(tests.sum()) / closed_s,
            "one_by_one": one, "served_over_one_by_one": None if one is None else S / one["value"],
            "oracle_equal": check,
            "oracle_check": "the first bucket of the committed fixture (%d requests) by SHA-256" % len(check_ids)
            if check_ids else None}


# --------------------------------------------------------------- clique search
def run_clique(args):
    """The k-clique question on the 4096 batching graphs: the search alone on
    each input graph, against the batched kernelization followed by the search
    on each kernel (same answers: every k-clique survives); the oracle's
    search on a sample of the input graphs (parity and CPU time)."""
    import torch

    from oracle import find_clique
    from paper_2212_00574_amd import inputs
    from paper_2212_00574_amd.binding import Batch, BatchKernelizer, Kernelizer, kz_gen_bitset
    dev = torch.device("cuda", 0)
    kz = Kernelizer(0)
    specs = inputs.config4_specs(args.seed)
    shapes = [(int(sp.sizes.sum()), int(((sp.sizes + 63) // 64).sum()), sp.k) for sp in specs]
    b = Batch.allocate(shapes, dev)
    planted = []
    for i, sp in enumerate(specs):
        d = b.desc[i]
        a, o = int(d["row_offset"]), int(d["vertex_offset"])
        pl = inputs.config4_graph(sp, args.seed, i).planted
        planted.append(pl)
        kz_gen_bitset(kz.ctx, sp.sizes, sp.p, args.seed, i, pl, b.rows[a:].data_ptr(), int(d["row_words"]),
                      b.colour[o:].data_ptr(), None)
    torch.cuda.synchronize()
    views = []
    for i in range(b.G):
        d = b.desc[i]
        n, R = int(d["n"]), int(d["row_words"])
        a, o = int(d["row_offset"]), int(d["vertex_offset"])
        views.append((b.rows[a:a + n * R].view(n, R), b.colour[o:o + n], int(d["k"]), b.vmask[o:o + n],
                      b.emask[a:a + n * R].view(n, R)))

    def search(kernel):
        out, nodes = [], 0
        for rows, col, k, vm, em in views:
            cl, r = kz.find_clique(em, col, k, vm) if kernel else kz.find_clique(rows, col, k)
            out.append(cl)
            nodes += r["nodes"]
        torch.cuda.synchronize()
        return [c.cpu().numpy() for c in out], nodes

    for rows, col, k, vm, em in views[:16]:   # warm-up
        kz.find_clique(rows, col, k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    raw, raw_nodes = search(False)
    raw_s = time.perf_counter() - t0
    bk = BatchKernelizer(kz)
    bk.run(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bk.run(b)
    torch.cuda.synchronize()
    kern_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    ker, ker_nodes = search(True)
    ksearch_s = time.perf_counter() - t0
    same = all(np.array_equal(x, y) for x, y in zip(raw, ker))
    found = sum(int(x[0] >= 0) for x in raw)

    def search_threads(nthreads):
        """The same searches from nthreads host threads, each with a context
        and a stream of its own (each call still blocks its own thread)."""
        import concurrent.futures as cf
        kzs = [Kernelizer(0) for _ in range(nthreads)]
        streams = [torch.cuda.Stream(dev) for _ in range(nthreads)]
        got = [None] * len(views)

        def work(t):
            with torch.cuda.stream(streams[t]):
                for i in range(t, len(views), nthreads):
                    rows, col, k, _, _ = views[i]
                    got[i] = kzs[t].find_clique(rows, col, k, stream=streams[t])[0]
            streams[t].synchronize()

        t0 = time.perf_counter()
        with cf.ThreadPoolExecutor(nthreads) as ex:
            list(ex.map(work, range(nthreads)))
        el = time.perf_counter() - t0
        answers = [c.cpu().numpy() for c in got]
        for k_ in kzs:
            k_.close()
        return el, all(np.array_equal(x, y) for x, y in zip(raw, answers))

    concurrent = {}
    for nt in (4, 8):
        el, eq = search_threads(nt)
        concurrent["threads_%d" % nt] = {"value": b.G / el, "seconds": round(el, 4), "same_answers": eq}
        say("clique: %d threads, search only %.3f s, same answers %s" % (nt, el, eq))
    # oracle on a sample of the input graphs
    sample = list(range(0, b.G, 128))
    ok = True
    t_or = 0.0
    for i in sample:
        g = inputs.config4_graph(specs[i], args.seed, i)
        rows, col, lay = g.bitset()
        adj = inputs.unpack_rows(rows, lay).astype(np.uint8)
        t0 = time.perf_counter()
        ref, _ = find_clique(adj, col, specs[i].k)
        t_or += time.perf_counter() - t0
        ok = ok and ((ref is None and raw[i][0] < 0) or (ref is not None and raw[i].tolist() == ref.tolist()))
    out = {"metric": "k-clique answers/s on the 4096 batching graphs", "unit": "graphs/s",
           "config": {"workload": "clique: " + WORKLOADS["clique"], "graphs": b.G, "seed": args.seed,
                      "planted": int(sum(p is not None for p in planted))},
           "found": found,
           "search_only": {"value": b.G / raw_s, "seconds": round(raw_s, 4), "nodes": raw_nodes},
           "kernel_then_search": {"value": b.G / (kern_s + ksearch_s), "seconds": round(kern_s + ksearch_s, 4),
                                  "kernelize_seconds": round(kern_s, 4), "search_seconds": round(ksearch_s, 4),
                                  "nodes": ker_nodes},
           "same_answers": same,
           "concurrent_callers": concurrent,
           "oracle_equal": ok,
           "oracle_check": "the class-order search of the oracle on every 128th input graph (%d graphs)" % len(sample),
           "cpu_baseline": {"value": len(sample) / t_or if t_or else None, "unit": "graphs/s", "cores": 1,
                            "kind": "oracle", "sample": "every 128th of the 4096 input graphs (%d), search only, "
                                                        "%.3f s" % (len(sample), t_or), "host": host_info()},
           "note": "one blocking kz_find_clique call per graph (a readback each); kernelization is one batched "
                   "launch for all 4096 graphs"}
    say("clique: %d found; search only %.3f s (%d nodes); kernel + search %.3f s (%d nodes)"
        % (found, raw_s, raw_nodes, kern_s + ksearch_s, ker_nodes))
    kz.close()
    return out


# --------------------------------------------------------------- more colours than the clique size
def run_colours(args):
    """The 4096 batching graphs with clique size max(1, k-2) below their k
    colour classes: batched time (median of three launches after a warm-up)
    against the same batch at clique size k, parity with the oracle's O3 on
    every 16th graph, and the oracle's time on those."""
    import torch

    from oracle import fixpoint_rows
    from paper_2212_00574_amd import inputs
    from paper_2212_00574_amd.binding import Batch, BatchKernelizer, Kernelizer, kz_gen_bitset
    dev = torch.device("cuda", 0)
    kz = Kernelizer(0)
    specs = inputs.config4_specs(args.seed)
    shapes = [(int(sp.sizes.sum()), int(((sp.sizes + 63) // 64).sum()), sp.k) for sp in specs]
    b = Batch.allocate(shapes, dev)
    for i, sp in enumerate(specs):
        d = b.desc[i]
        a, o = int(d["row_offset"]), int(d["vertex_offset"])
        kz_gen_bitset(kz.ctx, sp.sizes, sp.p, args.seed, i, inputs.config4_graph(sp, args.seed, i).planted,
                      b.rows[a:].data_ptr(), int(d["row_words"]), b.colour[o:].data_ptr(), None)
    torch.cuda.synchronize()
    bk = BatchKernelizer(kz)

    def timed():
        bk.run(b)
        torch.cuda.synchronize()
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            bk.run(b)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        return float(np.median(ts))

    plain_ms = timed()
    for i, sp in enumerate(specs):
        b.desc[i]["clique"] = max(1, sp.k - 2)
    b.desc_dev.copy_(torch.from_numpy(b.desc.view(np.uint8)))
    ms = timed()
    res = b.read_results()
    ok, t_or, sample = True, 0.0, list(range(0, b.G, 16))
    for i in sample:
        sp = specs[i]
        rows, col, _ = inputs.config4_graph(sp, args.seed, i).bitset()
        t0 = time.perf_counter()
        ref = fixpoint_rows(rows, col, sp.k, clique=max(1, sp.k - 2))
        t_or += time.perf_counter() - t0
        vm, em = b.masks(i)
        r = res[i]
        ok = ok and (int(r["rounds"]) == ref["rounds"] and int(r["edge_tests"]) == ref["edge_tests"]
                     and np.array_equal(vm, ref["vmask"]) and np.array_equal(em, ref["emask"]))
    out = {"metric": "batched graphs/s, clique size k-2 below k colour classes", "value": b.G / (ms / 1e3),
           "unit": "graphs/s", "ms_per_batch": round(ms, 3),
           "config": {"workload": "colours: " + WORKLOADS["colours"], "graphs": b.G, "seed": args.seed},
           "same_batch_clique_k": {"ms_per_batch": round(plain_ms, 3), "value": b.G / (plain_ms / 1e3)},
           "surviving_edges": int(res["surviving_edges"].sum()), "mean_rounds": float(res["rounds"].mean()),
           "oracle_equal": ok, "oracle_check": "O3 with the same clique size on every 16th graph (%d)" % len(sample),
           "cpu_baseline": {"value": len(sample) / t_or if t_or else None, "unit": "graphs/s", "cores": 1,
                            "kind": "oracle", "sample": "every 16th graph, %.2f s" % t_or, "host": host_info()},
           "note": "host timer around each launch of kz_kernelize_batch (no graph capture)"}
    say("colours: %.2f ms per batch at clique k-2 (%.2f ms at clique k), oracle equal %s" % (ms, plain_ms, ok))
    kz.close()
    return out


# --------------------------------------------------------------- struction
def run_struction(args):
    """Struction (section 4.1) of one random graph: plan + build time (median
    of three after a warm-up), the output's bytes over that time against the
    HBM peak, parity with the oracle's G' (every word), and the oracle's time."""
    import torch

    from oracle import struction
    from paper_2212_00574_amd import inputs
    from paper_2212_00574_amd.binding import Kernelizer
    kz = Kernelizer(0)
    rng = np.random.default_rng(np.random.SeedSequence([args.seed, 0x5354]))
    n, p = 1000, 0.1
    a = (rng.random((n, n)) < p).astype(np.uint8)
    a = np.triu(a, 1)
    adj = a + a.T
    rows = torch.from_numpy(inputs.dense_to_rows(adj).view(np.int64)).to(kz.device)
    kz.struction(rows, 0)
    torch.cuda.synchronize()
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        out, mp, res = kz.struction(rows, 0)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    ms = float(np.median(times))
    out_bytes = float(out.numel() * 8 + mp.numel() * 4)
    t0 = time.perf_counter()
    ref, rmap = struction(adj, 0)
    cpu_s = time.perf_counter() - t0
    equal = (np.array_equal(mp.cpu().numpy(), rmap)
             and np.array_equal(out.cpu().numpy().view(np.uint64), inputs.dense_to_rows(ref)))
    gbps = out_bytes / (ms / 1e3) / 1e9
    result = {"metric": "struction build time", "value": round(ms, 4), "unit": "ms", "higher_is_better": False,
              "config": {"workload": "struction: " + WORKLOADS["struction"], "n": n, "p": p, "pivot": 0,
                         "nodes": res["nodes"], "a_nodes": res["a_nodes"], "c_nodes": res["c_nodes"],
                         "seed": args.seed},
              "roofline": {"kernel": "k_st_rows (with plan, map and compression)", "bound": "hbm",
                           "achieved": round(gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                           "frac": round(gbps / HBM_PEAK_GBPS, 4), "traffic": None,
                           "bytes": "G' rows and node map written (n' * ceil(n'/64) * 8 + 8 n')",
                           "note": "whole blocking call (two readbacks) over the output bytes"},
              "oracle_equal": bool(equal),
              "cpu_baseline": {"value": round(cpu_s * 1e3, 1), "unit": "ms", "cores": 1, "kind": "oracle",
                               "sample": "the whole graph (dense n' x n' bytes), one core", "host": host_info()}}
    say("struction: n' = %d, %.3f ms (%.1f GB/s), oracle %.2f s, equal %s" % (res["nodes"], ms, gbps, cpu_s, equal))
    kz.close()
    return result


# --------------------------------------------------------------- colouring
def run_colouring(args):
    """Jones-Plassmann colouring of two uncoloured random graphs: whole-call
    time (median of three after a warm-up), rounds and colours; the smaller
    graph's colours against the oracle's, with the oracle's time."""
    import torch

    from oracle import colour_jp
    from paper_2212_00574_amd import inputs
    from paper_2212_00574_amd.binding import Kernelizer
    kz = Kernelizer(0)
    out = {}
    for i, (n, p) in enumerate(((3000, 0.3), (20000, 0.05))):
        rng = np.random.default_rng(np.random.SeedSequence([args.seed, 0x4A50, i]))
        dense = np.zeros((n, n), np.uint8)
        for v0 in range(0, n, 2048):       # the upper triangle by blocks of rows, then mirrored
            blk = rng.random((min(2048, n - v0), n), dtype=np.float32) < p
            dense[v0:v0 + blk.shape[0]] = np.triu(blk, v0 + 1)
        dense |= dense.T
        rows = inputs.dense_to_rows(dense)
        pri = rng.integers(0, 2**64, size=n, dtype=np.uint64)
        t_rows = torch.from_numpy(rows.view(np.int64)).to(kz.device)
        t_pri = torch.from_numpy(pri.view(np.int64)).to(kz.device)
        col, res = kz.colour_jp(t_rows, n, t_pri)
        torch.cuda.synchronize()
        times = []
        for _ in range(3):
            t0 = time.perf_counter()
            col, res = kz.colour_jp(t_rows, n, t_pri)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
        ms = float(np.median(times))
        entry = {"n": n, "p": p, "ms": round(ms, 3), "rounds": res["rounds"], "colours": res["colours"],
                 "us_per_round": round(ms * 1e3 / max(res["rounds"], 1), 2)}
        if n <= 5000:
            t0 = time.perf_counter()
            ref, rounds, nc = colour_jp(dense, pri)
            entry["oracle_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
            entry["oracle_equal"] = bool(np.array_equal(col.cpu().numpy(), ref) and rounds == res["rounds"])
        say("colouring: n %d p %.2f: %.2f ms, %d rounds, %d colours%s" % (
            n, p, ms, res["rounds"], res["colours"],
            ", oracle %.0f ms, equal %s" % (entry["oracle_ms"], entry["oracle_equal"]) if "oracle_ms" in entry else ""))
        out["n%d" % n] = entry
    kz.close()
    return {"metric": "colouring time", "value": out["n20000"]["ms"], "unit": "ms", "higher_is_better": False,
            "config": {"workload": "colouring: " + WORKLOADS["colouring"], "seed": args.seed},
            "graphs": out, "oracle_equal": out["n3000"].get("oracle_equal"),
            "note": "each round is two launches and one readback: launch-latency bound (us_per_round)"}


# --------------------------------------------------------------- dominance
def run_dom(args, cpu_proc=None):
    """Dominance reductions (section 4.3) on the ten evaluation graphs, both
    modes: per-graph times (median of up to three calls after one warm-up;
    each call runs the whole fixpoint and reads the counts back), parity with
    the oracle's full-size fixture, and the oracle's times on a sample."""
    import hashlib

    import torch

    from paper_2212_00574_amd import inputs
    from paper_2212_00574_amd.binding import KZ_DOM_EDGE, KZ_DOM_VERTEX, Kernelizer
    kz = Kernelizer(0)
    fx = golden("dom_seed%d.json" % args.seed)
    ref = {(r["mode"], r["n"]): r for r in fx["graphs"]} if fx else {}
    graphs = {}
    for n in DOM_SIZES:
        rows = inputs.dense_to_rows(inputs.dominance_graph(n, args.seed)).view(np.int64)
        graphs[n] = torch.from_numpy(rows).to(kz.device)
    torch.cuda.synchronize()
    out = {"metric": "dominance fixpoint time on the ten evaluation graphs", "unit": "ms", "higher_is_better": False,
           "config": {"workload": "dom: " + WORKLOADS["dom"], "sizes": DOM_SIZES, "seed": args.seed},
           "bound": "latency: a sweep is a chain of dependent steps (each step's tests run on one workgroup); "
                    "no HBM or ALU roof applies"}
    equal = bool(ref)
    reps = max(1, min(args.steps, 3))
    for name, mode in (("vertex", KZ_DOM_VERTEX), ("edge", KZ_DOM_EDGE)):
        per = {}
        for n, rows in graphs.items():
            times = []
            for rep in range(reps + 1):
                t0 = time.perf_counter()
                vm, em, r = kz.dominance(rows, mode)
                t1 = time.perf_counter()
                if rep:
                    times.append((t1 - t0) * 1e3)
            h = hashlib.sha256()
            h.update(vm.cpu().numpy().astype(np.uint8).tobytes())
            h.update(em.cpu().numpy().view(np.uint64).astype("<u8").tobytes())
            h.update(np.array([r["sweeps"], r["deleted_vertices"], r["deleted_edges"], r["events"]], "<i8").tobytes())
            rec = ref.get((name, n))
            if rec is None or rec["sha256"] != h.hexdigest():
                equal = False
            per[n] = {"ms": round(float(np.median(times)), 4), "sweeps": r["sweeps"],
                      "deleted_vertices": r["deleted_vertices"], "deleted_edges": r["deleted_edges"],
                      "edges": r["input_edges"]}
        out[name] = {"total_ms": round(sum(v["ms"] for v in per.values()), 3), "graphs": per}
        say("dom %s: %.2f ms for the ten graphs" % (name, out[name]["total_ms"]))
    out["oracle_equal"] = equal
    out["oracle_check"] = "SHA-256 of vmask || surviving rows || counts against tests/golden/dom_seed%d.json" % args.seed
    cpu = None
    if cpu_proc is not None:
        proc, core = cpu_proc
        o, err = proc.communicate(timeout=900)
        if proc.returncode == 0:
            d = json.loads(o.strip().splitlines()[-1])
            v_s = sum(d["vertex"].values())
            e_s = sum(d["edge"].values())
            e_gpu = sum(out["edge"]["graphs"][int(n)]["ms"] for n in d["edge"]) / 1e3
            cpu = {"value": round(v_s * 1e3, 3), "unit": "ms (vertex mode, ten graphs)", "cores": 1, "kind": "oracle",
                   "edge_mode_ms": round(e_s * 1e3, 1),
                   "sample": "vertex mode on all ten graphs; edge mode on n = %s only (%.1f s; the GPU takes %.1f ms "
                             "on the same five); pinned to cpu %d" % (", ".join(map(str, DOM_CPU_EDGE_SIZES)),
                                                                      e_s, e_gpu * 1e3, core),
                   "edge_gpu_speedup_on_sample": round(e_s / e_gpu, 1) if e_gpu else None,
                   "vertex_gpu_speedup": round(v_s / (out["vertex"]["total_ms"] / 1e3), 2),
                   "host": host_info()}
        else:
            say("dominance cpu child failed:", err[-1000:])
    out["cpu_baseline"] = cpu
    kz.close()
    return out


# --------------------------------------------------------------- main
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
    w = "c3a" if args.workload == "headline" else args.workload
    cpu_proc = dom_proc = None
    if not args.no_cpu_baseline and w in ("c1", "c2", "c3a", "c3b"):
        cpu_proc = start_cpu_child(w, args.seed)
    if not args.no_cpu_baseline and (w == "dom" or args.workload == "headline"):
        dom_proc = start_dom_cpu_child(args.seed)
    if w == "c4":
        out = run_batch(args)
    elif w == "c5":
        out = run_serve(args)
    elif w == "dom":
        out = run_dom(args, dom_proc)
    elif w == "clique":
        out = run_clique(args)
    elif w == "struction":
        out = run_struction(args)
    elif w == "colours":
        out = run_colours(args)
    elif w == "colouring":
        out = run_colouring(args)
    else:
        # serving first: its streams then take hardware queues before the
        # other workloads' streams do (a stream that shares the running
        # session launch's queue waits for that launch)
        serve = run_serve(args) if args.workload == "headline" else None
        out = run_single(args, w, cpu_proc)
        if args.workload == "headline":
            out["batch"] = run_batch(args)
            out["serve"] = serve
            out["dominance"] = run_dom(args, dom_proc)
            out["clique"] = run_clique(args)
            out["struction"] = run_struction(args)
            out["colours"] = run_colours(args)
            out["colouring"] = run_colouring(args)
    out.setdefault("n_gpus", 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
