"""Writes the full-size parity fixtures from the CPU oracle (calls only
``oracle/`` for results and ``paper_2212_00574_amd.inputs`` for the seeded
graphs).  Run from the repository root:

    python tests/golden/make_golden.py [c3a|c4|c5|dom ...] [--procs 8]

Every graph's record is the SHA-256 digest of

    vmask (n bytes) || emask (n * row_words little-endian uint64 words, the
    bit-row layout) || int64 LE [rounds, surviving vertices, surviving edges,
    exact-worklist edge tests]

as the oracle's O3 (synchronous rounds on bit rows, pinned against O1 in
tests/test_oracle.py) computes them.  To keep the fixtures small, the
digests of consecutive graphs are grouped in buckets: a bucket's hash is
the SHA-256 of its graphs' digests in order, stored with the graphs' ids
and summed counts.  The GPU tests compute the same digests from the
library's outputs and compare bucket by bucket.

Workloads (seed 0):
  c3a  k=20 classes x 1000 vertices, p=0.3 (one graph);
  c4   the 4096 batching graphs (k~U{4..16}, s_c~U{8..128}, p~U[0.2,0.8],
       10% planted cliques), buckets of 64 graphs;
  c5   of the 50,000 served requests: every request with n <= 5000, a
       seeded 2% of the others and the 100 largest, buckets of 256.
  dom  the dominance reductions (section 4.3) on the thesis's ten evaluation
       sizes n = 100, 300, ..., 1900 (inputs.dominance_graph, seed 0), vertex
       and edge mode; per graph and mode the SHA-256 of
           vmask (n bytes) || surviving adjacency as plain bit rows (n *
           ceil(n/64) little-endian uint64 words) || int64 LE [sweeps,
           deleted vertices, deleted edges, events]
       (events: steps that deleted nodes, or deleted edges), from
       oracle.dom_vertex / oracle.dom_edge.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import dom_edge, dom_vertex, fixpoint_rows  # noqa: E402
from paper_2212_00574_amd import inputs  # noqa: E402

SEED = 0
C4_BUCKET, C5_BUCKET = 64, 256


def digest(vmask, emask, rounds, sv, se, tests) -> bytes:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(vmask, np.uint8).tobytes())
    h.update(np.ascontiguousarray(emask).astype("<u8", copy=False).tobytes())
    h.update(np.array([rounds, sv, se, tests], "<i8").tobytes())
    return h.digest()


def c5_coverage(specs, seed=SEED):
    """Ids of the covered requests, ascending: n <= 5000, a seeded 2% of the
    rest, and the 100 largest (by n, then id)."""
    n = np.array([s.n for s in specs])
    small = set(np.nonzero(n <= 5000)[0].tolist())
    rest = np.nonzero(n > 5000)[0]
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x4356]))
    pick = set(rng.choice(rest, size=int(round(0.02 * len(rest))), replace=False).tolist()) if len(rest) else set()
    largest = set(sorted(range(len(specs)), key=lambda i: (-n[i], i))[:100])
    return sorted(small | pick | largest)


def _one(task):
    kind, gid = task
    if kind == "c3a":
        g = inputs.config3a(SEED)
        k = 20
    elif kind == "c4":
        spec = inputs.config4_specs(SEED)[gid]
        g = inputs.config4_graph(spec, SEED, gid)
        k = spec.k
    else:
        spec = _C5[gid]
        g = inputs.make_graph(spec.sizes, spec.p, seed=SEED, gid=gid, shuffle=False)
        k = spec.k
    rows, col, lay = g.bitset()
    r = fixpoint_rows(rows, col, k)
    assert r["status"] == 0, (kind, gid, r["status"])
    d = digest(r["vmask"], r["emask"], r["rounds"], r["surv_vertices"], r["surv_edges"], r["edge_tests"])
    return gid, d, r["rounds"], r["edge_tests"], r["surv_vertices"], r["surv_edges"], int(rows.shape[0])


_C5 = None
DOM_SIZES = list(range(100, 2000, 200))


def dom_digest(vmask, adj, sweeps, dv, de, events) -> bytes:
    n = adj.shape[0]
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(vmask, np.uint8).tobytes())
    h.update(inputs.dense_to_rows(adj).astype("<u8", copy=False).tobytes())
    h.update(np.array([sweeps, dv, de, events], "<i8").tobytes())
    assert n == len(vmask)
    return h.digest()


def _dom_one(task):
    mode, n = task
    adj = inputs.dominance_graph(n, SEED)
    t0 = time.time()
    if mode == "vertex":
        out, alive, st = dom_vertex(adj)
        d = dom_digest(alive, out, st["sweeps"], st["deleted_vertices"], st["deleted_edges"], st["steps"])
        rec = {"sweeps": st["sweeps"], "deleted_vertices": st["deleted_vertices"],
               "deleted_edges": st["deleted_edges"], "events": st["steps"]}
    else:
        out, st = dom_edge(adj)
        d = dom_digest(np.ones(n, np.uint8), out, st["sweeps"], 0, st["deleted_edges"], st["deleted_edges"])
        rec = {"sweeps": st["sweeps"], "deleted_vertices": 0, "deleted_edges": st["deleted_edges"],
               "events": st["deleted_edges"]}
    rec.update(mode=mode, n=n, edges=int(adj.sum()) // 2, sha256=d.hex(), oracle_s=round(time.time() - t0, 3))
    return rec


def buckets(results, size):
    out = []
    for b0 in range(0, len(results), size):
        part = results[b0:b0 + size]
        h = hashlib.sha256()
        for r in part:
            h.update(r[1])
        out.append({"ids": [int(r[0]) for r in part] if size > 64 else [int(part[0][0]), int(part[-1][0])],
                    "hash": h.hexdigest(), "rounds": int(sum(r[2] for r in part)),
                    "max_rounds": int(max(r[2] for r in part)), "edge_tests": int(sum(r[3] for r in part)),
                    "surv_vertices": int(sum(r[4] for r in part)), "surv_edges": int(sum(r[5] for r in part))})
    return out


def main():
    global _C5
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="*", default=["c3a", "c4", "c5"])
    ap.add_argument("--procs", type=int, default=8)
    args = ap.parse_args()
    for which in args.which:
        t0 = time.time()
        if which == "c3a":
            (gid, d, rounds, tests, sv, se, n), = [_one(("c3a", 0))]
            doc = {"workload": "c3a: k=20 classes x 1000 vertices (n=20000), p=0.3, uint64 bit rows", "seed": SEED,
                   "sha256": d.hex(), "rounds": rounds, "edge_tests": tests, "surv_vertices": sv,
                   "surv_edges": se, "n": n}
        elif which == "c4":
            tasks = [("c4", i) for i in range(4096)]
            with mp.get_context("fork").Pool(args.procs) as pool:
                res = pool.map(_one, tasks, chunksize=16)
            doc = {"workload": "c4: 4096 graphs, k~U{4..16}, class sizes~U{8..128}, p~U[0.2,0.8], "
                               "10% planted k-clique, uint64 bit rows", "seed": SEED, "graphs": 4096,
                   "bucket": C4_BUCKET, "buckets": buckets(res, C4_BUCKET)}
        elif which == "c5":
            _C5 = inputs.config5_specs(SEED)
            ids = c5_coverage(_C5)
            # largest first so the pool's tail is short; results re-sorted by id
            order = sorted(ids, key=lambda i: -_C5[i].n)
            with mp.get_context("fork").Pool(args.procs) as pool:
                res = sorted(pool.imap_unordered(_one, [("c5", i) for i in order], chunksize=1))
            doc = {"workload": "c5: served requests, n log-uniform [200,20000], k~U{5..30} near-equal classes, "
                               "p~U[0.1,0.9]; coverage: every request with n <= 5000, a seeded 2% of the rest, "
                               "the 100 largest", "seed": SEED, "requests": 50000, "covered": len(ids),
                   "bucket": C5_BUCKET, "buckets": buckets(res, C5_BUCKET)}
        elif which == "dom":
            tasks = sorted([(m, n) for m in ("vertex", "edge") for n in DOM_SIZES], key=lambda t: -t[1])
            with mp.get_context("fork").Pool(args.procs) as pool:
                res = pool.map(_dom_one, tasks, chunksize=1)
            res.sort(key=lambda r: (r["mode"], r["n"]))
            doc = {"workload": "dominance (section 4.3) on the ten evaluation sizes n = 100..1900, "
                               "m = n(n-5)/2, path plus skewed edges (inputs.dominance_graph)", "seed": SEED,
                   "graphs": res}
        else:
            raise SystemExit("unknown workload " + which)
        path = os.path.join(HERE, "%s_seed%d.json" % (which, SEED))
        with open(path, "w") as f:
            json.dump(doc, f, separators=(",", ":") if which == "c5" else (", ", ": "))
            f.write("\n")
        print("%s: %.1f s -> %s" % (which, time.time() - t0, path), flush=True)


if __name__ == "__main__":
    main()
