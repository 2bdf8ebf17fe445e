"""Pure-Python set-based references for tiny graphs (test infrastructure only).

Independent of ``kz_oracle.c``: these work on Python sets built straight from
an edge list, so they pin the C oracle rather than re-run it.

* ``colour_index_vertex`` / ``colour_index_edge`` -- the two colour indices of
  thesis section 4.2 (the vertex index and the edge index that follow
  Definition 4.2.1), counted over Python sets.
* ``sync_rounds`` -- the pruning rules (vertex index below k-1, edge index
  below k-2) applied in synchronous rounds until nothing changes.
* ``greatest_stable`` -- the result defined without any rule order: the
  largest pair (V', E') such that every vertex of V' has an E'-neighbour in
  every other class and every edge of E' has a common E'-neighbour in every
  third class.  Found by exhaustive search over all edge subsets, so only for
  graphs with a handful of edges.  Rule application can only remove elements
  outside every such pair and stops at a pair of that kind, so the fixpoint
  of the rules must equal it.
"""
from __future__ import annotations

from itertools import combinations


def _adj(n, edges):
    nb = [set() for _ in range(n)]
    for u, v in edges:
        nb[u].add(v)
        nb[v].add(u)
    return nb


def colour_index_vertex(nb, colour, v):
    return len({colour[w] for w in nb[v]})


def colour_index_edge(nb, colour, u, v):
    return len({colour[w] for w in nb[u] & nb[v]})


def sync_rounds(n, edges, colour, k):
    """(alive vertices, alive edges as frozensets, rounds)."""
    V = set(range(n))
    E = {frozenset(e) for e in edges}
    rounds = 0
    while True:
        nb = _adj(n, [tuple(e) for e in E])
        fv = {v for v in V if colour_index_vertex(nb, colour, v) < k - 1}
        fe = set()
        for e in E:
            u, v = tuple(e)
            if colour_index_edge(nb, colour, u, v) < k - 2:
                fe.add(e)
        if not fv and not fe:
            return V, E, rounds
        V -= fv
        E = {e for e in E if e not in fe and not (e & fv)}
        rounds += 1


def _cond_vertex(nb, colour, k, v):
    have = {colour[w] for w in nb[v]}
    return all(c in have for c in range(k) if c != colour[v])


def _cond_edge(nb, colour, k, u, v):
    have = {colour[w] for w in nb[u] & nb[v]}
    return all(c in have for c in range(k) if c not in (colour[u], colour[v]))


def greatest_stable(n, edges, colour, k, max_edges=16):
    """Union of all stable pairs, by exhaustive search over edge subsets."""
    edges = [tuple(sorted(e)) for e in edges]
    if len(edges) > max_edges:
        raise ValueError("exhaustive search limited to %d edges" % max_edges)
    bestV, bestE = set(), set()
    for r in range(len(edges) + 1):
        for sub in combinations(edges, r):
            nb = _adj(n, sub)
            Vp = {v for v in range(n) if _cond_vertex(nb, colour, k, v)}
            if not all(u in Vp and v in Vp for u, v in sub):
                continue
            if not all(_cond_edge(nb, colour, k, u, v) for u, v in sub):
                continue
            bestV |= Vp
            bestE |= {frozenset(e) for e in sub}
    return bestV, bestE


def kcliques(n, edges, colour, k):
    """All k-cliques with one vertex per colour class, as sorted vertex tuples."""
    nb = _adj(n, edges)
    classes = [[v for v in range(n) if colour[v] == c] for c in range(k)]
    out = []

    def rec(c, pick):
        if c == k:
            out.append(tuple(sorted(pick)))
            return
        for v in classes[c]:
            if all(v in nb[p] for p in pick):
                rec(c + 1, pick + [v])

    if n and all(classes):
        rec(0, [])
    return out
