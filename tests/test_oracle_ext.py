"""Pins of the dominance oracle (section 4.3, Definitions 4.3.1 and 4.3.2,
Algorithms 1 and 2 as read in oracle/kz_oracle_ext.c), checked against
hand derivations and against properties the definitions fix -- not against
a second copy of the same loops:

* hand-derived results on small graphs, including ones where the order of
  the sweep decides the result (twins, a deletion that enables a later one);
* the clique number never changes (brute force over vertex subsets): every
  single deletion trades a for b inside any clique through it;
* the result is a fixpoint: no surviving vertex (edge) is dominated, checked
  with Python sets;
* vertex dominance leaves an induced subgraph, edge dominance a spanning
  subgraph, both symmetric, and the counts add up.
"""
import itertools

import numpy as np
import pytest

from oracle import dom_edge, dom_vertex


def graph(n, edges):
    a = np.zeros((n, n), np.uint8)
    for u, v in edges:
        a[u, v] = a[v, u] = 1
    return a


def edges_of(a):
    n = a.shape[0]
    return {(u, v) for u in range(n) for v in range(u + 1, n) if a[u, v]}


def omega(a, alive=None):
    n = a.shape[0]
    vs = [v for v in range(n) if alive is None or alive[v]]
    best = 1 if vs else 0
    for r in range(2, len(vs) + 1):
        found = any(all(a[x, y] for x, y in itertools.combinations(c, 2)) for c in itertools.combinations(vs, r))
        if not found:
            break
        best = r
    return best


def nbrs(a, v):
    return {w for w in range(a.shape[0]) if a[v, w]}


def random_graph(rng, n, p):
    a = (rng.random((n, n)) < p).astype(np.uint8)
    a = np.triu(a, 1)
    return a + a.T


# ---------------------------------------------------------------- vertex
def test_vertex_cycle_of_four():
    # step b=0 deletes 2 (N(2) = {1,3} = N(0)); only then is N(3) = {0} a
    # subset of N(1) = {0}, so step b=1 deletes 3
    a, alive, st = dom_vertex(graph(4, [(0, 1), (1, 2), (2, 3), (3, 0)]))
    assert alive.tolist() == [1, 1, 0, 0]
    assert edges_of(a) == {(0, 1)}
    assert st == {"sweeps": 1, "deleted_vertices": 2, "deleted_edges": 3, "steps": 2}


def test_vertex_twins_keep_the_first():
    # 0 and 1 both see only 2: step b=0 deletes 1, and 0 survives (deleting
    # both at once would lose every edge of the graph)
    a, alive, st = dom_vertex(graph(3, [(0, 2), (1, 2)]))
    assert alive.tolist() == [1, 0, 1]
    assert edges_of(a) == {(0, 2)}
    assert st["deleted_vertices"] == 1 and st["deleted_edges"] == 1


def test_vertex_dominated_by_a_later_node():
    # step b=0 finds nothing (N(1) = {2,3}, N(3) = {1}); step b=1 deletes
    # a=0 < b (N(0) = {2} is in N(1)); then N(2) = {1} and step b=2 deletes
    # its twin 3 (N(3) = {1})
    a, alive, st = dom_vertex(graph(4, [(0, 2), (1, 2), (1, 3)]))
    assert alive.tolist() == [0, 1, 1, 0]
    assert edges_of(a) == {(1, 2)}
    assert st["steps"] == 2


def test_vertex_edgeless_and_star_and_complete():
    _, alive, st = dom_vertex(graph(4, []))
    assert alive.tolist() == [1, 0, 0, 0] and st["deleted_edges"] == 0
    _, alive, _ = dom_vertex(graph(4, [(0, 1), (0, 2), (0, 3)]))
    assert alive.tolist() == [1, 1, 0, 0]
    k4 = graph(4, itertools.combinations(range(4), 2))
    a, alive, st = dom_vertex(k4)
    assert alive.all() and (a == k4).all() and st["sweeps"] == 0


# ---------------------------------------------------------------- edge
def test_edge_path_of_three():
    # a=0, u=1, b=2: N(0) & N(1) is empty, so {1,2} dominates {0,1}
    a, st = dom_edge(graph(3, [(0, 1), (1, 2)]))
    assert edges_of(a) == {(1, 2)}
    assert st == {"sweeps": 1, "deleted_edges": 1}


def test_edge_k4_minus_an_edge():
    # a=0: u=2, b=1: N(0) & N(2) = {3} is in N(1) -> delete {0,2};
    #      u=3, b=1: N(0) & N(3) is now empty -> delete {0,3};
    # the triangle {1,2,3} has no non-adjacent b left
    a, st = dom_edge(graph(4, [(0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]))
    assert edges_of(a) == {(1, 2), (1, 3), (2, 3)}
    assert st["deleted_edges"] == 2


def test_edge_triangle_and_complete_are_kept():
    for n in (3, 5):
        k = graph(n, itertools.combinations(range(n), 2))
        a, st = dom_edge(k)
        assert (a == k).all() and st["deleted_edges"] == 0


# ---------------------------------------------------------------- properties
def vertex_fixpoint_ok(a, alive):
    n = a.shape[0]
    for b in range(n):
        for x in range(n):
            if x == b or not alive[b] or not alive[x] or a[x, b]:
                continue
            if nbrs(a, x) <= nbrs(a, b):
                return False
    return True


def edge_fixpoint_ok(a):
    n = a.shape[0]
    for x in range(n):
        for u in nbrs(a, x):
            common = nbrs(a, x) & nbrs(a, u)
            for b in nbrs(a, u):
                if b != x and not a[x, b] and common <= nbrs(a, b):
                    return False
    return True


@pytest.mark.parametrize("seed", range(6))
def test_vertex_properties(seed):
    rng = np.random.default_rng(seed)
    multi = 0
    for _ in range(40):
        n = int(rng.integers(1, 10))
        g = random_graph(rng, n, float(rng.uniform(0.15, 0.9)))
        a, alive, st = dom_vertex(g)
        assert (a == a.T).all() and not a.diagonal().any()
        keep = alive.astype(bool)
        assert (a[np.ix_(keep, keep)] == g[np.ix_(keep, keep)]).all()   # induced subgraph
        assert not a[~keep].any()
        assert st["deleted_vertices"] == n - int(keep.sum())
        assert st["deleted_edges"] == len(edges_of(g)) - len(edges_of(a))
        assert keep.sum() >= min(n, 1)
        assert omega(a, alive) == omega(g)
        assert vertex_fixpoint_ok(a, alive)
        multi += st["sweeps"] >= 2
    assert multi >= 1   # some graph needs a second sweep


@pytest.mark.parametrize("seed", range(6))
def test_edge_properties(seed):
    rng = np.random.default_rng(100 + seed)
    for _ in range(40):
        n = int(rng.integers(2, 10))
        g = random_graph(rng, n, float(rng.uniform(0.2, 0.9)))
        a, st = dom_edge(g)
        assert (a == a.T).all() and not a.diagonal().any()
        assert not (a & ~g.astype(bool)).any()                              # only deletions
        assert st["deleted_edges"] == len(edges_of(g)) - len(edges_of(a))
        assert omega(a) == omega(g)
        assert edge_fixpoint_ok(a)


def test_edge_second_sweeps_reach_the_fixpoint():
    # a deletion late in a sweep can make an earlier edge dominated (about 2 %
    # of these graphs); the fixpoint check must still hold for them
    rng = np.random.default_rng(7)
    multi = 0
    for _ in range(600):
        n = int(rng.integers(3, 12))
        g = random_graph(rng, n, float(rng.uniform(0.2, 0.9)))
        a, st = dom_edge(g)
        if st["sweeps"] >= 2:
            multi += 1
            assert edge_fixpoint_ok(a) and omega(a) == omega(g)
    assert multi >= 3


# ---------------------------------------------------------------- clique search
from oracle import FMT_DENSE, OracleGraph, find_clique  # noqa: E402


def coloured_graph(rng, sizes, p, plant=False):
    sizes = [int(s) for s in sizes]
    n = sum(sizes)
    colour = np.repeat(np.arange(len(sizes), dtype=np.int32), sizes)
    a = (rng.random((n, n)) < p).astype(np.uint8)
    a = np.triu(a, 1)
    a = a + a.T
    a[colour[:, None] == colour[None, :]] = 0
    if plant and all(sizes):
        pick = [int(rng.integers(0, s)) + int(np.sum(sizes[:c])) for c, s in enumerate(sizes)]
        for x, y in itertools.combinations(pick, 2):
            a[x, y] = a[y, x] = 1
    return a, colour


def brute_smallest(a, colour, k, alive=None):
    classes = [[v for v in range(a.shape[0]) if colour[v] == c and (alive is None or alive[v])] for c in range(k)]
    for tup in itertools.product(*classes):     # lexicographic in class order
        if all(a[x, y] for x, y in itertools.combinations(tup, 2)):
            return list(tup)
    return None


@pytest.mark.parametrize("seed", range(5))
def test_clique_search_is_the_brute_force_smallest(seed):
    rng = np.random.default_rng(300 + seed)
    found = 0
    for _ in range(60):
        k = int(rng.integers(1, 5))
        sizes = rng.integers(1, 5, size=k)
        a, colour = coloured_graph(rng, sizes, float(rng.uniform(0.3, 0.95)), plant=bool(rng.random() < 0.3))
        alive = (rng.random(a.shape[0]) < 0.85).astype(np.uint8) if rng.random() < 0.5 else None
        got, nodes = find_clique(a, colour, k, alive)
        ref = brute_smallest(a, colour, k, alive)
        assert (got is None) == (ref is None)
        if ref is not None:
            found += 1
            assert got.tolist() == ref
            assert nodes >= k
    assert found >= 20


def test_clique_search_agrees_with_the_clique_count():
    # OracleGraph.kcliques (pinned by closed forms and itertools in
    # test_oracle.py) counts k-cliques; the search finds one iff it is > 0
    rng = np.random.default_rng(17)
    for _ in range(40):
        k = int(rng.integers(2, 6))
        sizes = rng.integers(2, 8, size=k)
        a, colour = coloured_graph(rng, sizes, float(rng.uniform(0.2, 0.8)))
        og = OracleGraph(FMT_DENSE, a.shape[0], k, colour, adj=a)
        count = og.kcliques()[0]
        got, _ = find_clique(a, colour, k)
        assert (got is not None) == (count > 0)
        if got is not None:
            assert len(set(colour[got].tolist())) == k
            assert all(a[x, y] for x, y in itertools.combinations(got.tolist(), 2))


def test_clique_search_complete_multipartite_and_live_mask():
    sizes = [3, 1, 4, 2]
    a, colour = coloured_graph(np.random.default_rng(0), sizes, 1.0)
    got, nodes = find_clique(a, colour, 4)
    assert got.tolist() == [0, 3, 4, 8] and nodes == 4          # first vertex of every class
    alive = np.ones(a.shape[0], np.uint8)
    alive[[0, 4]] = 0
    got, _ = find_clique(a, colour, 4, alive)
    assert got.tolist() == [1, 3, 5, 8]
    alive[3] = 0                                                 # class 1 emptied
    assert find_clique(a, colour, 4, alive)[0] is None
    assert find_clique(a, colour, 1)[0].tolist() == [0]


# ---------------------------------------------------------------- struction
from oracle import struction  # noqa: E402


def test_struction_hand_example():
    # pivot 0: A = {1}; B = {2, 3, 4} with edges 23, 24, 34 -> C = c(2,3),
    # c(2,4), c(3,4); 1 ~ c(2,3) (1 ~ 2 and 1 ~ 3); c(2,3) ~ c(2,4) (same
    # first vertex, 3 ~ 4); omega: 3 in G ({1,2,3}, {2,3,4}), 2 in G'
    g = graph(5, [(0, 1), (1, 2), (2, 3), (3, 4), (2, 4), (1, 3)])
    out, mp = struction(g, 0)
    assert mp.tolist() == [[1, -1], [2, 3], [2, 4], [3, 4]]
    assert edges_of(out) == {(0, 1), (1, 2)}
    assert omega(g) == 3 and omega(out) == 2


@pytest.mark.parametrize("seed", range(6))
def test_struction_lowers_the_clique_number_by_one(seed):
    rng = np.random.default_rng(500 + seed)
    for _ in range(40):
        n = int(rng.integers(1, 9))
        g = random_graph(rng, n, float(rng.uniform(0.1, 0.95)))
        p = int(rng.integers(0, n))
        out, mp = struction(g, p)
        A = [v for v in range(n) if g[p, v]]
        B = [v for v in range(n) if v != p and not g[p, v]]
        inner = [(x, y) for x in B for y in B if x < y and g[x, y]]
        assert mp.tolist() == [[a, -1] for a in A] + [list(e) for e in inner]
        assert (out == out.T).all() and not out.diagonal().any()
        assert omega(out) == omega(g) - 1          # Theorem 1


# ---- upstream legal colouring (Jones and Plassmann, SIAM J. Sci. Comput.
# 14(3), 1993), pinned by hand derivations, a closed form on complete
# graphs, and the properties the algorithm guarantees, checked with Python
# sets rather than a second copy of its loops.
from oracle import colour_jp  # noqa: E402


def test_jp_path_and_star_by_hand():
    # path 0-1-2-3, priorities 10 40 20 30: round 1 takes 1 (beats 0 and 2)
    # and 3 (beats 2), both colour 0; round 2 takes 0 and 2, colour 1
    col, rounds, nc = colour_jp(graph(4, [(0, 1), (1, 2), (2, 3)]), np.array([10, 40, 20, 30], np.uint64))
    assert col.tolist() == [1, 0, 1, 0] and rounds == 2 and nc == 2
    # star with the centre lowest: the leaves first (colour 0), then the centre
    col, rounds, nc = colour_jp(graph(5, [(0, i) for i in range(1, 5)]), np.array([1, 5, 4, 3, 2], np.uint64))
    assert col.tolist() == [1, 0, 0, 0, 0] and rounds == 2 and nc == 2
    # the centre highest: it alone first, then every leaf in round 2
    col, rounds, nc = colour_jp(graph(5, [(0, i) for i in range(1, 5)]), np.array([9, 5, 4, 3, 2], np.uint64))
    assert col.tolist() == [0, 1, 1, 1, 1] and rounds == 2 and nc == 2
    # triangle 0-1-2 and a pendant 3 on 2, priorities 3 2 1 4: round 1 takes
    # 0 (beats 1, 2) and 3 (beats 2): colour 0 each; round 2 takes 1 (its
    # uncoloured neighbour 2 is lower): colour 1; round 3 takes 2: neighbours
    # hold 0, 1, 0, so colour 2
    col, rounds, nc = colour_jp(graph(4, [(0, 1), (1, 2), (0, 2), (2, 3)]), np.array([3, 2, 1, 4], np.uint64))
    assert col.tolist() == [0, 1, 2, 0] and rounds == 3 and nc == 3


def test_jp_complete_graph_colours_are_ranks():
    """On K_n each round takes the one uncoloured vertex with the largest
    key, which takes the next colour: colour(v) is v's rank by key,
    largest first (ties in priority broken by the larger index)."""
    rng = np.random.default_rng(5)
    for n in (1, 2, 7, 40):
        a = np.ones((n, n), np.uint8) - np.eye(n, dtype=np.uint8)
        pri = rng.integers(0, 2**63, size=n, dtype=np.uint64)
        col, rounds, nc = colour_jp(a, pri)
        order = sorted(range(n), key=lambda v: (int(pri[v]), v), reverse=True)
        assert [int(col[v]) for v in order] == list(range(n))
        assert rounds == n and nc == n
        col, _, _ = colour_jp(a, np.zeros(n, np.uint64))          # equal priorities: by index
        assert col.tolist() == list(range(n - 1, -1, -1))


def test_jp_edgeless_and_empty():
    col, rounds, nc = colour_jp(np.zeros((6, 6), np.uint8), np.arange(6, dtype=np.uint64))
    assert col.tolist() == [0] * 6 and rounds == 1 and nc == 1
    col, rounds, nc = colour_jp(np.zeros((0, 0), np.uint8), np.zeros(0, np.uint64))
    assert len(col) == 0 and rounds == 0 and nc == 0


def jp_random(n, p, seed):
    rng = np.random.default_rng(seed)
    a = np.triu((rng.random((n, n)) < p).astype(np.uint8), 1)
    a = a | a.T
    return a, rng.integers(0, 2**64, size=n, dtype=np.uint64)


def test_jp_properties_on_random_graphs():
    """A legal colouring; greedy (a vertex of colour c has neighbours of
    every colour below c); at most max degree + 1 colours; the vertex with
    the largest key takes colour 0; and relabelling the vertices (with
    their priorities) relabels the colours the same way."""
    for n, p, seed in ((30, 0.2, 1), (60, 0.5, 2), (80, 0.1, 3), (50, 0.9, 4)):
        a, pri = jp_random(n, p, seed)
        col, rounds, nc = colour_jp(a, pri)
        nbrs = [set(np.nonzero(a[v])[0].tolist()) for v in range(n)]
        for v in range(n):
            assert all(col[u] != col[v] for u in nbrs[v])
            assert set(range(col[v])) <= {int(col[u]) for u in nbrs[v]}
        assert nc == col.max() + 1 <= max(len(s) for s in nbrs) + 1
        top = max(range(n), key=lambda v: (int(pri[v]), v))
        assert col[top] == 0
        perm = np.random.default_rng(seed + 10).permutation(n)
        inv = np.argsort(perm)
        # vertex i of the relabelled graph is old vertex perm[i]; keys
        # (priority, index) must order the same, so the priorities are
        # distinct here (ties would be broken by the new indices)
        assert len(set(pri.tolist())) == n
        col2, rounds2, nc2 = colour_jp(a[np.ix_(perm, perm)], pri[perm])
        assert np.array_equal(col2[inv], col) and rounds2 == rounds and nc2 == nc
