"""Seeded synthetic inputs: legally coloured graphs in the library's three formats.

This module only *generates* graphs.  It holds none of the kernelization
arithmetic (no colour index, no test, no removal), so the CPU oracle's tests
and the GPU path can both take their inputs from here without sharing any of
the method.

Edge draws.  Every inter-class vertex pair {a, b} (class-major slot ids, a < b)
of graph ``gid`` under ``seed`` is an edge iff

    h = splitmix64(splitmix64((seed << 32) | gid) ^ ((a << 32) | b))  <  floor(p * 2**64)

where ``splitmix64`` is the output function of Steele, Lea and Flood's
SplitMix64 generator ("Fast splittable pseudorandom number generators",
OOPSLA 2014): add the golden-gamma increment 0x9E3779B97F4A7C15, then two
xor-shift-multiply rounds (30, 0xBF58476D1CE4E5B9; 27, 0x94D049BB133111EB)
and a final xor-shift by 31.  The draw is a pure function of (seed, gid, a, b),
so any slice of a graph can be regenerated anywhere.  Pairs inside one colour
class are never edges (the colouring is legal by construction).

Everything else (planted vertices, class sizes, vertex order, per-graph
parameters) comes from ``numpy.random.default_rng(SeedSequence([...]))``.

Formats (the slot order is class-major: class 0's vertices first, then
class 1's, ... ; within a class, increasing slot id):

* DENSE  -- ``adj`` uint8 [n, n] in a seeded random vertex order, 0/1,
  symmetric, zero diagonal; ``colour`` int32 [n] in that order.
* BITSET -- ``rows`` uint64 [n, R] in slot order.  Segment c of a row starts
  at word ``segoff[c]`` and has ``W_c = ceil(s_c / 64)`` words; bit j of the
  segment (word j // 64, bit j % 64, little-endian) is adjacency to the
  j-th vertex of class c.  Padding bits are zero.  ``colour`` is the sorted
  class-major colour vector.
* CSR    -- ``row_ptr`` int64 [n+1], ``col_idx`` int32 [nnz], both edge
  directions, column ids strictly increasing within a row, in a seeded random
  vertex order.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from fractions import Fraction

import numpy as np

U64 = np.uint64
_GAMMA = U64(0x9E3779B97F4A7C15)
_M1 = U64(0xBF58476D1CE4E5B9)
_M2 = U64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1


def splitmix64(x):
    """SplitMix64 output function on uint64 (scalar or array); wraps mod 2**64."""
    x = np.asarray(x, dtype=U64)
    with np.errstate(over="ignore"):
        z = x + _GAMMA
        z = (z ^ (z >> U64(30))) * _M1
        z = (z ^ (z >> U64(27))) * _M2
        return z ^ (z >> U64(31))


def splitmix64_int(x: int) -> int:
    """Pure-Python SplitMix64 output function (reference for the vectorised one)."""
    z = (x + 0x9E3779B97F4A7C15) & _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def edge_threshold(p: float) -> int:
    """floor(p * 2**64) from the exact binary value of the float p, clamped to [0, 2**64 - 1]."""
    if p <= 0.0:
        return 0
    t = Fraction(p) * (1 << 64)
    return min(int(t), _MASK64)


def graph_base(seed: int, gid: int) -> int:
    if not (0 <= seed < (1 << 32) and 0 <= gid < (1 << 32)):
        raise ValueError("seed and graph id must fit in 32 bits")
    return splitmix64_int((seed << 32) | gid)


def pair_is_edge(seed: int, gid: int, a: int, b: int, p: float) -> bool:
    """Scalar edge draw for slot pair {a, b} (no class check)."""
    lo, hi = (a, b) if a < b else (b, a)
    return splitmix64_int(graph_base(seed, gid) ^ ((lo << 32) | hi)) < edge_threshold(p)


def _draw_block(base: int, thr: int, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Edge draws for the outer product a[:,None] x b[None,:] (slot ids); bool."""
    A = a.astype(U64)[:, None]
    B = b.astype(U64)[None, :]
    lo = np.minimum(A, B)
    hi = np.maximum(A, B)
    key = U64(base) ^ ((lo << U64(32)) | hi)
    return splitmix64(key) < U64(thr)


# --------------------------------------------------------------------------- layout
@dataclass
class ClassLayout:
    sizes: np.ndarray            # int64 [k]
    offsets: np.ndarray          # int64 [k+1]  first slot of each class
    words: np.ndarray            # int64 [k]    W_c
    segoff: np.ndarray           # int64 [k+1]  first word of each segment
    n: int = field(init=False)
    k: int = field(init=False)
    R: int = field(init=False)

    def __post_init__(self):
        self.n = int(self.offsets[-1])
        self.k = int(len(self.sizes))
        self.R = int(self.segoff[-1])


def class_layout(sizes) -> ClassLayout:
    sizes = np.asarray(sizes, dtype=np.int64)
    offsets = np.zeros(len(sizes) + 1, np.int64)
    offsets[1:] = np.cumsum(sizes)
    words = (sizes + 63) // 64
    segoff = np.zeros(len(sizes) + 1, np.int64)
    segoff[1:] = np.cumsum(words)
    return ClassLayout(sizes, offsets, words, segoff)


def sorted_colour(sizes) -> np.ndarray:
    return np.repeat(np.arange(len(sizes), dtype=np.int32), np.asarray(sizes, np.int64))


# --------------------------------------------------------------------------- generation
@dataclass
class Graph:
    """One generated graph.  ``slot_adj``-free: formats are produced on demand."""
    sizes: np.ndarray
    p: float
    seed: int
    gid: int
    planted: np.ndarray | None   # slot ids, one per class (or None)
    order: np.ndarray            # caller vertex id -> slot id (DENSE/CSR order)

    @property
    def k(self) -> int:
        return int(len(self.sizes))

    @property
    def n(self) -> int:
        return int(np.sum(self.sizes))

    @property
    def layout(self) -> ClassLayout:
        return class_layout(self.sizes)

    # -- slot-order boolean rows (block of rows) ------------------------------
    def slot_rows(self, r0: int, r1: int) -> np.ndarray:
        """bool [r1-r0, n]: adjacency of slots r0..r1-1 to every slot."""
        lay = self.layout
        n = lay.n
        col = sorted_colour(self.sizes)
        a = np.arange(r0, r1, dtype=np.int64)
        b = np.arange(n, dtype=np.int64)
        blk = _draw_block(graph_base(self.seed, self.gid), edge_threshold(self.p), a, b)
        blk &= col[r0:r1, None] != col[None, :]
        if self.planted is not None and len(self.planted):
            pl = np.asarray(self.planted, np.int64)
            inblk = pl[(pl >= r0) & (pl < r1)]
            for s in inblk:
                others = pl[pl != s]
                blk[s - r0, others] = True
        return blk

    def dense_slot(self) -> np.ndarray:
        return self.slot_rows(0, self.n).astype(np.uint8)

    # -- formats ---------------------------------------------------------------
    def bitset(self, chunk: int = 512) -> tuple[np.ndarray, np.ndarray, ClassLayout]:
        """(rows uint64 [n, R], colour int32 [n] sorted, layout)."""
        lay = self.layout
        rows = np.zeros((lay.n, max(lay.R, 0)), dtype=np.uint64)
        for r0 in range(0, lay.n, chunk):
            r1 = min(lay.n, r0 + chunk)
            rows[r0:r1] = pack_rows(self.slot_rows(r0, r1), lay)
        return rows, sorted_colour(self.sizes), lay

    def dense(self) -> tuple[np.ndarray, np.ndarray]:
        """(adj uint8 [n, n], colour int32 [n]) in the caller vertex order."""
        slot = self.dense_slot()
        o = self.order
        adj = np.ascontiguousarray(slot[np.ix_(o, o)])
        return adj, sorted_colour(self.sizes)[o].astype(np.int32)

    def csr(self) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
        adj, colour = self.dense()
        rp, ci = dense_to_csr(adj)
        return rp, ci, colour


def pack_rows(slot_bool: np.ndarray, lay: ClassLayout) -> np.ndarray:
    """bool [r, n] slot-order rows -> uint64 [r, R] class-segmented bit rows."""
    r = slot_bool.shape[0]
    out = np.zeros((r, lay.R), dtype=np.uint64)
    for c in range(lay.k):
        s = int(lay.sizes[c])
        w = int(lay.words[c])
        if w == 0:
            continue
        seg = np.zeros((r, 64 * w), dtype=bool)
        seg[:, :s] = slot_bool[:, lay.offsets[c]:lay.offsets[c] + s]
        packed = np.packbits(seg, axis=1, bitorder="little")
        out[:, lay.segoff[c]:lay.segoff[c] + w] = packed.view("<u8").reshape(r, w)
    return out


def unpack_rows(rows: np.ndarray, lay: ClassLayout) -> np.ndarray:
    """uint64 [r, R] -> bool [r, n] slot-order rows (padding dropped)."""
    r = rows.shape[0]
    out = np.zeros((r, lay.n), dtype=bool)
    for c in range(lay.k):
        s = int(lay.sizes[c])
        w = int(lay.words[c])
        if w == 0:
            continue
        seg = np.ascontiguousarray(rows[:, lay.segoff[c]:lay.segoff[c] + w]).astype("<u8")
        bits = np.unpackbits(seg.view(np.uint8).reshape(r, 8 * w), axis=1, bitorder="little")
        out[:, lay.offsets[c]:lay.offsets[c] + s] = bits[:, :s].astype(bool)
    return out


def dense_to_csr(adj: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    n = adj.shape[0]
    nz_r, nz_c = np.nonzero(adj)
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, nz_r + 1, 1)
    rp = np.cumsum(rp)
    return rp.astype(np.int64), nz_c.astype(np.int32)


def csr_to_dense(n: int, rp: np.ndarray, ci: np.ndarray) -> np.ndarray:
    adj = np.zeros((n, n), np.uint8)
    rows = np.repeat(np.arange(n), np.diff(rp))
    adj[rows, ci] = 1
    return adj


def _rng(*key: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(list(key)))


def make_graph(sizes, p: float, seed: int = 0, gid: int = 0, plant: bool = False,
               shuffle: bool = True) -> Graph:
    """A legally coloured random graph with the given class sizes.

    ``plant`` forces a k-clique through one uniformly drawn vertex per class.
    ``shuffle`` draws the caller vertex order used by the DENSE and CSR formats.
    """
    sizes = np.asarray(sizes, np.int64)
    lay = class_layout(sizes)
    rng = _rng(seed, gid, 0x504C)
    planted = None
    if plant:
        if np.any(sizes == 0):
            raise ValueError("cannot plant a clique with an empty class")
        planted = np.array([lay.offsets[c] + rng.integers(0, sizes[c]) for c in range(len(sizes))],
                           dtype=np.int64)
    order = _rng(seed, gid, 0x4F52).permutation(lay.n) if shuffle else np.arange(lay.n)
    return Graph(sizes, float(p), int(seed), int(gid), planted, order.astype(np.int64))


# --------------------------------------------------------------------------- the five workloads
def config1(seed: int = 0) -> Graph:
    """Small: k=4 classes x 25 vertices, inter-class p=0.5, DENSE uint8 input."""
    return make_graph([25] * 4, 0.5, seed=seed, gid=0)


def config2(seed: int = 0) -> Graph:
    """Mid: k=10 x 300 (n=3000), p=0.6, one planted 10-clique, BITSET input."""
    return make_graph([300] * 10, 0.6, seed=seed, gid=0, plant=True, shuffle=False)


def config3a(seed: int = 0) -> Graph:
    """Large dense: k=20 x 1000 (n=20000), p=0.3, BITSET input."""
    return make_graph([1000] * 20, 0.3, seed=seed, gid=0, shuffle=False)


@dataclass
class SparseGraph:
    n: int
    k: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    colour: np.ndarray
    sizes: np.ndarray


def make_sparse(n: int, k: int, m: int, seed: int = 0) -> SparseGraph:
    """Uneven classes (multinomial over k) and m distinct inter-class pairs drawn uniformly."""
    rng = _rng(seed, 0, 0x5350)
    sizes = rng.multinomial(n, [1.0 / k] * k).astype(np.int64)
    colour = np.repeat(np.arange(k, dtype=np.int32), sizes)
    colour = colour[rng.permutation(n)]
    have = np.zeros(0, dtype=np.int64)
    while have.size < m:
        need = m - have.size
        draw = rng.integers(0, n, size=(int(need * 1.2) + 64, 2), dtype=np.int64)
        a, b = draw[:, 0], draw[:, 1]
        ok = colour[a] != colour[b]
        a, b = a[ok], b[ok]
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        key = lo * n + hi
        have = np.concatenate([have, key])
        _, first = np.unique(have, return_index=True)
        have = have[np.sort(first)]          # keep first occurrences, in draw order
    have = have[:m]
    lo, hi = have // n, have % n
    src = np.concatenate([lo, hi])
    dst = np.concatenate([hi, lo])
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, src + 1, 1)
    rp = np.cumsum(rp)
    return SparseGraph(n, k, rp, dst.astype(np.int32), colour.astype(np.int32), sizes)


def config3b(seed: int = 0) -> SparseGraph:
    """Large sparse: k=30, n=100000, multinomial classes, 2.5M inter-class edges (avg degree 50), CSR."""
    return make_sparse(100_000, 30, 2_500_000, seed=seed)


@dataclass
class BatchSpec:
    k: int
    sizes: np.ndarray
    p: float
    plant: bool


def config4_specs(seed: int = 0, graphs: int = 4096) -> list[BatchSpec]:
    """Batch: per graph k~U{4..16}, s_c~U{8..128}, density~U[0.2,0.8], planted clique w.p. 0.1."""
    rng = _rng(seed, 0, 0x4234)
    out = []
    for _ in range(graphs):
        k = int(rng.integers(4, 17))
        sizes = rng.integers(8, 129, size=k).astype(np.int64)
        p = float(rng.uniform(0.2, 0.8))
        plant = bool(rng.random() < 0.1)
        out.append(BatchSpec(k, sizes, p, plant))
    return out


def config4_graph(spec: BatchSpec, seed: int, gid: int) -> Graph:
    return make_graph(spec.sizes, spec.p, seed=seed, gid=gid, plant=spec.plant, shuffle=False)


@dataclass
class ServeSpec:
    n: int
    k: int
    sizes: np.ndarray
    p: float
    arrival_s: float


def config5_specs(seed: int = 0, requests: int = 50_000, rate_hz: float = 1000.0) -> list[ServeSpec]:
    """Serving: n log-uniform in [200, 20000], k~U{5..30}, near-equal classes, p~U[0.1,0.9], Poisson arrivals."""
    rng = _rng(seed, 0, 0x5356)
    out = []
    t = 0.0
    for _ in range(requests):
        n = int(round(np.exp(rng.uniform(np.log(200), np.log(20000)))))
        k = int(rng.integers(5, 31))
        base, extra = divmod(n, k)
        sizes = np.array([base + (1 if c < extra else 0) for c in range(k)], np.int64)
        p = float(rng.uniform(0.1, 0.9))
        t += float(rng.exponential(1.0 / rate_hz))
        out.append(ServeSpec(n, k, sizes, p, t))
    return out


# ---------------------------------------------------------------- dominance
# Uncoloured graphs for the dominance reductions.  The thesis evaluates them
# on ten saved random graphs of 100, 300, ..., 1900 vertices whose edge count
# is a fixed function of n (its table gives n(n-5)/2: 4750 at n = 100,
# 44250 at 300, ...), built by first laying a path through every vertex in
# order and then adding edges that are not uniformly random: some vertices
# tend to take more edges than others.  Recipe here (the thesis's files are
# not available): the path {i, i+1} is always present; vertex v gets a
# tendency t_v = u_v ** 2, u_v uniform on [0, 1); of the other pairs, the
# C(n,2) - m that stay absent are drawn without replacement with weight
# (1 - t_a)(1 - t_b) + 1e-3, so vertices with a high tendency keep more
# edges.  m defaults to n(n-5)/2 (clipped to [n-1, C(n,2)]).
def dominance_graph(n: int, seed: int = 0, m: int | None = None) -> np.ndarray:
    """Dense uint8 [n, n] adjacency (symmetric, zero diagonal)."""
    n = int(n)
    adj = np.zeros((n, n), np.uint8)
    if n < 2:
        return adj
    full = n * (n - 1) // 2
    m = full if m is None and n < 6 else (n * (n - 5) // 2 if m is None else int(m))
    m = min(max(m, n - 1), full)
    rng = _rng(0xD0, seed, n)
    t = rng.random(n) ** 2
    iu, ju = np.triu_indices(n, 1)
    off_path = ju != iu + 1
    a, b = iu[off_path], ju[off_path]
    absent = full - m
    keep = np.ones(a.size, bool)
    if absent > 0:
        w = (1.0 - t[a]) * (1.0 - t[b]) + 1e-3
        drop = rng.choice(a.size, size=absent, replace=False, p=w / w.sum())
        keep[drop] = False
    adj[a[keep], b[keep]] = 1
    adj[np.arange(n - 1), np.arange(1, n)] = 1
    return adj | adj.T


def dense_to_rows(adj: np.ndarray) -> np.ndarray:
    """Plain bit rows uint64 [n, ceil(n/64)] of a dense 0/1 adjacency (bit w % 64
    of word w // 64 of row v is adj[v, w])."""
    n = adj.shape[0]
    R = max((n + 63) // 64, 1)
    padded = np.zeros((n, R * 64), np.uint8)
    padded[:, :n] = adj
    bits = np.packbits(padded.reshape(n, R, 64)[:, :, ::-1], axis=2).reshape(n, R, 8)
    return bits[:, :, ::-1].copy().view("<u8").reshape(n, R)


def rows_to_dense(rows: np.ndarray, n: int) -> np.ndarray:
    """Inverse of dense_to_rows."""
    rows = np.ascontiguousarray(rows).view(np.uint64).reshape(n, -1)
    b = rows.view(np.uint8).reshape(n, -1, 8)[:, :, ::-1]
    bits = np.unpackbits(b, axis=2)[:, :, ::-1].reshape(n, -1)
    return bits[:, :n].astype(np.uint8)
