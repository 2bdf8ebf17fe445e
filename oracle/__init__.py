"""CPU oracle for iterated colour-index pruning -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The product library never loads it, and it
shares no code with the GPU path: the C file ``kz_oracle.c`` reads the
caller's arrays itself (see its header for the thesis passages it follows,
section 4.2 and Definition 4.2.1).

Functions and their pins (each is checked in ``tests/test_oracle.py`` against
something other than itself):

* ``OracleGraph.fixpoint`` (O1, synchronous rounds) -- pinned by the thesis's
  Figure 8 colour indices on a consistent completion (golden fixture), the
  k=2 / k=3 closed forms (k=3 kernel = union of triangles, checked against
  brute-force triangle enumeration), complete k-partite graphs, the
  index-inequality family (no k-clique yet nothing removed), brute-force
  k-clique inclusion, and, on tiny graphs, equality with the greatest stable
  subgraph found by exhaustive search over edge subsets (``setref``).
* ``OracleGraph.fixpoint_random_order`` (O2) -- pinned by agreeing with O1
  over many random orders and by the same exhaustive search.
* ``OracleGraph.ci_vertex`` / ``ci_edge`` -- pinned by the four colour
  indices the thesis prints for Figure 8.
* ``OracleGraph.kcliques`` -- pinned by closed-form clique counts of complete
  k-partite graphs (prod of class sizes) and by itertools enumeration.
* ``fixpoint_rows`` (O3, the synchronous rounds of O1 on plain bit rows, for
  graphs too large for O1's adjacency lists) -- pinned by equality with O1
  (masks, rounds, survivors, exact-worklist counts, validation statuses) on
  seeded graphs of every shape the tests use, and by the same closed forms:
  Figure 8's hand-derived fixpoint, the k=3 kernel = union of triangles,
  complete multipartite graphs and the index-inequality family.  With a
  clique size below the number of classes (``clique``): the clique-3 kernel
  of an m-coloured graph is the union of its triangles, the clique-2 kernel
  drops only isolated vertices, complete m-partite graphs keep everything,
  every vertex and edge of every clique-sized clique survives (brute force),
  kernels shrink as the clique size grows, and a hand case.
* ``witness_words`` (a measurement, not a result: the words a first-witness
  search reads over every (edge, third class) pair of the input) -- pinned
  by a pure-Python count on small graphs and by closed forms (complete
  multipartite graphs: one word per pair; a class emptied of common
  neighbours: its whole segment, counted as a pair without a witness).
* ``OracleGraph.failing`` -- vertex output pinned by Figure 8's round-1
  survivors (hand derivation); edge output pinned by the Figure 8 edges whose
  printed or derived index is below k-2 (all report 1), by complete
  multipartite graphs (no edge fails) and by the same graphs with one class
  emptied (every edge fails).
* ``OracleGraph.set_masks`` -- pinned by round trips through ``masks`` in
  all three formats, by resuming from the kernel (no round, invariant I2) and
  from the input (same result), and by rejecting one-way edges, edges at dead
  vertices, edges absent from the input and non-0/1 bytes.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import build_oracle

FMT_DENSE, FMT_BITSET, FMT_CSR = 0, 1, 2

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # KZ_ORACLE_LIB lets the mutation test load a copy of the oracle with a
    # planted mistake, to show that the pins catch it.
    lib = C.CDLL(os.environ.get("KZ_ORACLE_LIB") or build_oracle())
    vp, i32, i64, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
    lib.kzo_load.restype = vp
    lib.kzo_load.argtypes = [C.c_int, i32, vp, vp, i32, vp, vp, i64, vp, i32, C.POINTER(i32)]
    lib.kzo_free.argtypes = [vp]
    lib.kzo_reset.argtypes = [vp]
    lib.kzo_num_entries.restype = i64
    lib.kzo_num_entries.argtypes = [vp]
    lib.kzo_fixpoint.restype = C.c_int
    lib.kzo_fixpoint.argtypes = [vp, vp]
    lib.kzo_fixpoint_random_order.restype = C.c_int
    lib.kzo_fixpoint_random_order.argtypes = [vp, u64]
    lib.kzo_ci_vertex.restype = i32
    lib.kzo_ci_vertex.argtypes = [vp, i32]
    lib.kzo_ci_edge.restype = i32
    lib.kzo_ci_edge.argtypes = [vp, i32, i32]
    lib.kzo_kcliques.restype = i64
    lib.kzo_kcliques.argtypes = [vp, vp, vp]
    lib.kzo_get_masks.argtypes = [vp, vp, vp]
    lib.kzo_set_masks.restype = C.c_int
    lib.kzo_set_masks.argtypes = [vp, vp, vp]
    lib.kzo_failing.argtypes = [vp, vp, i64, vp, vp, vp, i64, vp]
    lib.kzo_fixpoint_rows.restype = C.c_int
    lib.kzo_fixpoint_rows.argtypes = [i32, i32, vp, vp, i32, vp, vp, vp]
    lib.kzo_fixpoint_rows_mk.restype = C.c_int
    lib.kzo_fixpoint_rows_mk.argtypes = [i32, i32, i32, vp, vp, i32, vp, vp, vp]
    lib.kzo_witness_words.restype = i64
    lib.kzo_witness_words.argtypes = [i32, i32, vp, vp, i32, C.POINTER(i64), C.POINTER(i64)]
    lib.kzo_dom_vertex.restype = C.c_int
    lib.kzo_dom_vertex.argtypes = [i32, vp, vp, vp]
    lib.kzo_dom_edge.restype = C.c_int
    lib.kzo_dom_edge.argtypes = [i32, vp, vp]
    lib.kzo_struction.restype = i64
    lib.kzo_struction.argtypes = [i32, vp, i32, vp, i64, vp]
    lib.kzo_find_clique.restype = C.c_int
    lib.kzo_find_clique.argtypes = [i32, vp, vp, i32, vp, vp, vp]
    lib.kzo_colour_jp.restype = C.c_int
    lib.kzo_colour_jp.argtypes = [i32, vp, vp, vp, C.POINTER(i32)]
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class OracleError(ValueError):
    def __init__(self, status):
        super().__init__("oracle rejected the input, status %d" % status)
        self.status = status


class OracleGraph:
    """One validated input graph held by the C oracle."""

    def __init__(self, fmt, n, k, colour, adj=None, rows=None, row_words=0,
                 row_ptr=None, col_idx=None):
        lib = _load()
        self.fmt, self.n, self.k = int(fmt), int(n), int(k)
        self._keep = []
        colour = np.ascontiguousarray(colour, dtype=np.int32)
        self._keep.append(colour)
        args = dict(adj=None, rows=None, rp=None, ci=None)
        nnz = 0
        if fmt == FMT_DENSE:
            args["adj"] = np.ascontiguousarray(adj, dtype=np.uint8)
        elif fmt == FMT_BITSET:
            args["rows"] = np.ascontiguousarray(rows, dtype=np.uint64)
        else:
            args["rp"] = np.ascontiguousarray(row_ptr, dtype=np.int64)
            args["ci"] = np.ascontiguousarray(col_idx, dtype=np.int32)
            nnz = int(args["ci"].size)
        self._keep += [a for a in args.values() if a is not None]
        self.row_words = int(row_words)
        st = C.c_int32(0)
        self._h = lib.kzo_load(self.fmt, self.n, _ptr(args["adj"]), _ptr(args["rows"]),
                               self.row_words, _ptr(args["rp"]), _ptr(args["ci"]), nnz,
                               _ptr(colour), self.k, C.byref(st))
        self.status = int(st.value)
        if not self._h:
            raise OracleError(self.status)
        self.nent = int(lib.kzo_num_entries(self._h))
        self._keep = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _load().kzo_free(h)
            self._h = None

    def reset(self):
        _load().kzo_reset(self._h)

    def fixpoint(self) -> dict:
        stats = np.zeros(5, np.int64)
        st = _load().kzo_fixpoint(self._h, _ptr(stats))
        if st:
            raise OracleError(st)
        return dict(rounds=int(stats[0]), equals_input=int(stats[1]), surv_vertices=int(stats[2]),
                    surv_edges=int(stats[3]), edge_tests=int(stats[4]))

    def fixpoint_random_order(self, seed: int):
        st = _load().kzo_fixpoint_random_order(self._h, C.c_uint64(seed & (2**64 - 1)))
        if st:
            raise OracleError(st)

    def ci_vertex(self, v: int) -> int:
        return int(_load().kzo_ci_vertex(self._h, int(v)))

    def ci_edge(self, u: int, v: int) -> int:
        return int(_load().kzo_ci_edge(self._h, int(u), int(v)))

    def _emask_buffer(self):
        if self.fmt == FMT_DENSE:
            return np.zeros((self.n, self.n), np.uint8)
        if self.fmt == FMT_BITSET:
            return np.zeros((self.n, self.row_words), np.uint64)
        return np.zeros(self.nent, np.uint8)

    def masks(self):
        vmask = np.zeros(self.n, np.uint8)
        emask = self._emask_buffer()
        _load().kzo_get_masks(self._h, _ptr(vmask), _ptr(emask))
        return vmask, emask

    def set_masks(self, vmask, emask) -> bool:
        vmask = np.ascontiguousarray(vmask, dtype=np.uint8)
        emask = np.ascontiguousarray(emask, dtype=self._emask_buffer().dtype)
        return _load().kzo_set_masks(self._h, _ptr(vmask), _ptr(emask)) == 0

    def kcliques(self):
        """(count, vin u8[n], ein u8[entries]) over the input graph's k-cliques."""
        vin = np.zeros(max(self.n, 1), np.uint8)
        ein = np.zeros(max(self.nent, 1), np.uint8)
        cnt = _load().kzo_kcliques(self._h, _ptr(vin), _ptr(ein))
        return int(cnt), vin[:self.n], ein[:self.nent]

    def failing(self, vs=(), us=(), ws=()):
        vs = np.ascontiguousarray(vs, dtype=np.int32)
        us = np.ascontiguousarray(us, dtype=np.int32)
        ws = np.ascontiguousarray(ws, dtype=np.int32)
        vf = np.zeros(max(vs.size, 1), np.uint8)
        ef = np.zeros(max(us.size, 1), np.uint8)
        _load().kzo_failing(self._h, _ptr(vs), vs.size, _ptr(vf), _ptr(us), _ptr(ws), us.size, _ptr(ef))
        return vf[:vs.size], ef[:us.size]


def _run(g: OracleGraph) -> dict:
    res = g.fixpoint()
    res["vmask"], res["emask"] = g.masks()
    res["status"] = 0
    return res


def _guard(fn):
    try:
        return _run(fn())
    except OracleError as e:
        return dict(status=e.status)


def kernelize_dense(adj, colour, k) -> dict:
    adj = np.asarray(adj)
    return _guard(lambda: OracleGraph(FMT_DENSE, adj.shape[0], k, colour, adj=adj))


def kernelize_bitset(rows, colour, k, row_words=None) -> dict:
    rows = np.asarray(rows)
    rw = rows.shape[1] if row_words is None else row_words
    return _guard(lambda: OracleGraph(FMT_BITSET, rows.shape[0], k, colour, rows=rows, row_words=rw))


def kernelize_csr(row_ptr, col_idx, colour, k) -> dict:
    n = len(row_ptr) - 1
    return _guard(lambda: OracleGraph(FMT_CSR, n, k, colour, row_ptr=row_ptr, col_idx=col_idx))


def fixpoint_rows(rows, colour, k, clique=None) -> dict:
    """O3 on class-major bit rows (the BITSET format): same result and
    counts as O1.  Returns the dict of ``kernelize_bitset`` (emask as uint64
    rows).  ``clique`` (default k) is the clique size when the k colour
    classes outnumber it: thresholds clique-1 and clique-2."""
    rows = np.ascontiguousarray(rows, dtype=np.uint64)
    colour = np.ascontiguousarray(colour, dtype=np.int32)
    n = int(colour.size)
    R = int(rows.shape[1]) if rows.ndim == 2 else 0
    if n and rows.shape[0] != n:
        raise ValueError("rows and colour disagree on n")
    vmask = np.zeros(n, np.uint8)
    emask = np.zeros((n, R), np.uint64)
    stats = np.zeros(5, np.int64)
    kk = int(k) if clique is None else int(clique)
    st = _load().kzo_fixpoint_rows_mk(n, int(k), kk, _ptr(colour), _ptr(rows) if rows.size else None, R,
                                      _ptr(vmask), _ptr(emask) if emask.size else None, _ptr(stats))
    if st:
        return dict(status=int(st))
    return dict(status=0, rounds=int(stats[0]), equals_input=int(stats[1]), surv_vertices=int(stats[2]),
                surv_edges=int(stats[3]), edge_tests=int(stats[4]), vmask=vmask, emask=emask)


def witness_words(rows, colour, k) -> dict:
    """{"words", "pairs", "no_witness"}: over every edge u < v of a valid
    bit-row input and every class other than the endpoints', the words read
    in order up to the first common neighbour (whole segment if none)."""
    rows = np.ascontiguousarray(rows, dtype=np.uint64)
    colour = np.ascontiguousarray(colour, dtype=np.int32)
    pairs, nowit = C.c_int64(0), C.c_int64(0)
    w = _load().kzo_witness_words(int(colour.size), int(k), _ptr(colour), _ptr(rows), int(rows.shape[1]),
                                  C.byref(pairs), C.byref(nowit))
    return {"words": int(w), "pairs": int(pairs.value), "no_witness": int(nowit.value)}


# ---- dominance (section 4.3), kz_oracle_ext.c
def _dense01(adj):
    a = np.ascontiguousarray(adj, dtype=np.uint8).copy()
    n = a.shape[0]
    assert a.shape == (n, n)
    return a, n


def dom_vertex(adj):
    """Sweeps of Algorithm 1 (Definition 4.3.1, read as documented in
    kz_oracle_ext.c) to a fixpoint.  Returns (adjacency after deletion,
    alive mask, stats dict)."""
    a, n = _dense01(adj)
    alive = np.zeros(n, np.uint8)
    st = np.zeros(4, np.int64)
    _load().kzo_dom_vertex(n, _ptr(a), _ptr(alive), _ptr(st))
    return a, alive, {"sweeps": int(st[0]), "deleted_vertices": int(st[1]), "deleted_edges": int(st[2]),
                      "steps": int(st[3])}


def dom_edge(adj):
    """Sweeps of Algorithm 2 (Definition 4.3.2, read as documented in
    kz_oracle_ext.c) to a fixpoint.  Returns (adjacency after deletion,
    stats dict)."""
    a, n = _dense01(adj)
    st = np.zeros(2, np.int64)
    _load().kzo_dom_edge(n, _ptr(a), _ptr(st))
    return a, {"sweeps": int(st[0]), "deleted_edges": int(st[1])}


# ---- k-clique search on a (kernelized) graph, kz_oracle_ext.c
def find_clique(adj, colour, k, alive=None):
    """The lexicographically smallest k-clique (class 0's vertex first) among
    the live vertices of a legally k-coloured dense graph: (clique int32[k]
    or None, nodes).  nodes counts the partial picks the plain class-order
    search extends (a measure, not a result)."""
    a = np.ascontiguousarray(adj, dtype=np.uint8)
    n = a.shape[0]
    col = np.ascontiguousarray(colour, dtype=np.int32)
    al = None if alive is None else np.ascontiguousarray(alive, dtype=np.uint8)
    out = np.zeros(max(int(k), 1), np.int32)
    nodes = np.zeros(1, np.int64)
    f = _load().kzo_find_clique(n, _ptr(a), _ptr(col), int(k), _ptr(al), _ptr(out), _ptr(nodes))
    if f < 0:
        raise MemoryError("oracle: allocation failed")
    return (out[:k].copy() if f else None), int(nodes[0])


# ---- struction (section 4.1), kz_oracle_ext.c
def struction(adj, pivot=0):
    """G' of Definition 4.1.1 around `pivot` (readings in kz_oracle_ext.c):
    (adjacency uint8 [n', n'], map int32 [n', 2]: (vertex, -1) for the
    pivot's neighbours A, (x, y) for the nodes c(x, y) of C)."""
    a = np.ascontiguousarray(adj, dtype=np.uint8)
    n = a.shape[0]
    lib = _load()
    npr = int(lib.kzo_struction(n, _ptr(a), int(pivot), None, 0, None))
    if npr < 0:
        raise ValueError("pivot outside the graph")
    out = np.zeros((max(npr, 1), max(npr, 1)), np.uint8)
    mp = np.zeros((max(npr, 1), 2), np.int32)
    got = int(lib.kzo_struction(n, _ptr(a), int(pivot), _ptr(out), npr, _ptr(mp)))
    assert got == npr
    return out[:npr, :npr].copy(), mp[:npr].copy()



# ---- upstream legal colouring (Jones-Plassmann), kz_oracle_ext.c
def colour_jp(adj, priority):
    """Jones and Plassmann's parallel greedy colouring of a dense graph with
    the given uint64 priorities (keys (priority[v], v)): (colour int32[n],
    rounds, number of colours)."""
    a = np.ascontiguousarray(adj, dtype=np.uint8)
    n = a.shape[0]
    pri = np.ascontiguousarray(priority, dtype=np.uint64)
    assert pri.shape == (n,)
    col = np.zeros(max(n, 1), np.int32)
    nc = C.c_int32(0)
    r = _load().kzo_colour_jp(n, _ptr(a), _ptr(pri), _ptr(col), C.byref(nc))
    if r < 0:
        raise RuntimeError("oracle: a colouring round took no vertex")
    return col[:n].copy(), int(r), int(nc.value)
