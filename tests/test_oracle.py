"""Pins for the CPU oracle (no GPU).  Each test checks the oracle against
something other than itself: the thesis's printed colour indices for its
Figure 8 (section 4.2), closed forms, brute force, or the order-free
definition of the result searched exhaustively."""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import (FMT_BITSET, FMT_CSR, FMT_DENSE, OracleError, OracleGraph,
                    kernelize_bitset, kernelize_csr, kernelize_dense, setref)
from paper_2212_00574_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

pytestmark = pytest.mark.filterwarnings("ignore")


def dense_from_edges(n, edges):
    adj = np.zeros((n, n), np.uint8)
    for u, v in edges:
        adj[u, v] = adj[v, u] = 1
    return adj


def edges_of(adj):
    u, v = np.nonzero(np.triu(adj, 1))
    return list(zip(u.tolist(), v.tolist()))


def run_dense(adj, colour, k):
    g = OracleGraph(FMT_DENSE, adj.shape[0], k, colour, adj=adj)
    res = g.fixpoint()
    vm, em = g.masks()
    return g, res, vm, em


def random_small(n_per_class, k, p, seed, plant=False):
    g = inputs.make_graph([n_per_class] * k, p, seed=seed, gid=7, plant=plant)
    adj, colour = g.dense()
    return adj, colour


# ----------------------------------------------------------------- Figure 8
def load_fig8():
    fx = json.load(open(os.path.join(GOLDEN, "figure8.json")))
    names = fx["vertices"]
    idx = {v: i for i, v in enumerate(names)}
    colour = np.array([fx["colour"][v] for v in names], np.int32)
    edges = [(idx[a], idx[b]) for a, b in fx["edges"]]
    return fx, idx, colour, dense_from_edges(len(names), edges)


def test_figure8_completion_is_consistent_with_stated_facts():
    fx, idx, colour, adj = load_fig8()
    kf = fx["known_facts"]
    for v in ("a", "d"):
        want = set(kf["neighbours_of_" + v])
        got = {n for n, i in idx.items() if adj[idx[v], i]}
        assert got == want
    for v, c in kf["colours"].items():
        assert colour[idx[v]] == c
    assert adj[idx["h"], idx["f"]] and adj[idx["i"], idx["f"]]


def test_figure8_colour_indices_match_paper():
    fx, idx, colour, adj = load_fig8()
    pv = fx["known_facts"]["paper_values"]
    g = OracleGraph(FMT_DENSE, len(idx), fx["k"], colour, adj=adj)
    assert g.ci_vertex(idx["a"]) == pv["ci_vertex_a"] == 2
    assert g.ci_vertex(idx["d"]) == pv["ci_vertex_d"] == 3
    assert g.ci_edge(idx["a"], idx["d"]) == pv["ci_edge_a_d"] == 0
    assert g.ci_edge(idx["h"], idx["i"]) == pv["ci_edge_h_i"] == 1
    assert g.ci_edge(idx["a"], idx["e"]) == -1          # not an edge
    nb = setref._adj(len(idx), edges_of(adj))
    assert setref.colour_index_vertex(nb, colour, idx["a"]) == 2
    assert setref.colour_index_edge(nb, colour, idx["h"], idx["i"]) == 1


def test_figure8_fixpoint_hand_derived():
    fx, idx, colour, adj = load_fig8()
    exp = fx["expected_fixpoint"]
    g, res, vm, em = run_dense(adj, colour, fx["k"])
    assert res["rounds"] == exp["rounds"] == 2
    assert res["equals_input"] == 0
    assert vm.sum() == 0 and em.sum() == 0
    # round-1 survivors: the vertices whose index reaches k-1
    r1 = {v for v, i in idx.items() if g.ci_vertex(i) >= fx["k"] - 1} if False else None
    g2 = OracleGraph(FMT_DENSE, len(idx), fx["k"], colour, adj=adj)
    vf, _ = g2.failing(vs=np.arange(len(idx)))
    survivors = {v for v, i in idx.items() if not vf[i]}
    assert survivors == set(exp["round1_surviving_vertices"])
    V, E = setref.greatest_stable(len(idx), edges_of(adj), colour, fx["k"])
    assert V == set() and E == set()


# ----------------------------------------------------------- closed forms
@pytest.mark.parametrize("seed", range(6))
def test_k2_closed_form(seed):
    adj, colour = random_small(12, 2, 0.15, seed)
    g, res, vm, em = run_dense(adj, colour, 2)
    deg = adj.sum(1)
    assert np.array_equal(em, adj)                       # no edge test applies at k=2
    assert np.array_equal(vm, (deg > 0).astype(np.uint8))
    assert res["rounds"] == (1 if (deg == 0).any() else 0)


def triangles(adj):
    n = adj.shape[0]
    tv, te = set(), set()
    for a, b, c in itertools.combinations(range(n), 3):
        if adj[a, b] and adj[b, c] and adj[a, c]:
            tv |= {a, b, c}
            te |= {(a, b), (b, c), (a, c)}
    return tv, te


@pytest.mark.parametrize("seed,p", [(s, p) for s in range(5) for p in (0.08, 0.2, 0.5)])
def test_k3_kernel_is_union_of_triangles(seed, p):
    adj, colour = random_small(9, 3, p, seed)
    g, res, vm, em = run_dense(adj, colour, 3)
    tv, te = triangles(adj)
    assert set(np.nonzero(vm)[0].tolist()) == tv
    assert set(edges_of(em)) == te
    # rounds: 0 if nothing goes; 2 if some vertex sees both other classes yet is in no triangle; else 1
    n = adj.shape[0]
    sees_both = [len({colour[w] for w in np.nonzero(adj[v])[0]}) == 2 for v in range(n)]
    if len(te) == len(edges_of(adj)) and len(tv) == n:
        want = 0
    elif any(sees_both[v] and v not in tv for v in range(n)):
        want = 2
    else:
        want = 1
    assert res["rounds"] == want


@pytest.mark.parametrize("k,s", [(2, 3), (3, 2), (4, 3), (5, 2), (6, 1)])
def test_complete_multipartite_is_its_own_kernel(k, s):
    colour = np.repeat(np.arange(k), s).astype(np.int32)
    adj = (colour[:, None] != colour[None, :]).astype(np.uint8)
    g, res, vm, em = run_dense(adj, colour, k)
    assert res["rounds"] == 0 and res["equals_input"] == 1
    assert np.array_equal(em, adj) and vm.all()
    cnt, vin, ein = g.kcliques()
    assert cnt == s ** k


@pytest.mark.parametrize("k", [2, 3, 4, 6])
def test_empty_class_empties_the_graph_in_one_round(k):
    colour = np.repeat(np.arange(k - 1), 3).astype(np.int32)   # class k-1 is empty
    adj = (colour[:, None] != colour[None, :]).astype(np.uint8)
    g, res, vm, em = run_dense(adj, colour, k)
    assert res["rounds"] == 1 and vm.sum() == 0 and em.sum() == 0


def index_inequality(k):
    """k classes x (k-1) vertices (c, i); (c,i)~(c',i') iff c != c' and i != i'."""
    verts = [(c, i) for c in range(k) for i in range(k - 1)]
    n = len(verts)
    adj = np.zeros((n, n), np.uint8)
    for a, (c, i) in enumerate(verts):
        for b, (d, j) in enumerate(verts):
            if c != d and i != j:
                adj[a, b] = 1
    return adj, np.array([c for c, _ in verts], np.int32)


@pytest.mark.parametrize("k", [4, 5, 6])
def test_index_inequality_family_keeps_everything_without_a_clique(k):
    adj, colour = index_inequality(k)
    g, res, vm, em = run_dense(adj, colour, k)
    assert g.kcliques()[0] == 0
    assert res["rounds"] == 0 and vm.all() and np.array_equal(em, adj)


def test_index_inequality_k3_collapses_in_two_rounds():
    adj, colour = index_inequality(3)
    g, res, vm, em = run_dense(adj, colour, 3)
    assert res["rounds"] == 2 and vm.sum() == 0 and em.sum() == 0


def test_trivial_sizes():
    # n = 0
    g = OracleGraph(FMT_DENSE, 0, 3, np.zeros(0, np.int32), adj=np.zeros((0, 0), np.uint8))
    r = g.fixpoint()
    assert r["rounds"] == 0 and r["equals_input"] == 1
    # k = 1: a legal 1-colouring has no edges; nothing is removed
    adj = np.zeros((4, 4), np.uint8)
    _, r, vm, em = run_dense(adj, np.zeros(4, np.int32), 1)
    assert r["rounds"] == 0 and vm.all()


# ---------------------------------------------------- soundness (brute force)
@pytest.mark.parametrize("seed", range(8))
def test_every_kclique_survives(seed):
    k = 3 + seed % 3
    adj, colour = random_small(6, k, 0.55, seed, plant=(seed % 2 == 0))
    g, res, vm, em = run_dense(adj, colour, k)
    cnt, vin, ein = g.kcliques()
    cl = setref.kcliques(adj.shape[0], edges_of(adj), colour, k)
    assert cnt == len(cl)
    for clique in cl:
        for v in clique:
            assert vm[v]
        for a, b in itertools.combinations(clique, 2):
            assert em[a, b] and em[b, a]
    assert np.all(vm >= vin)


def test_config1_cliques_survive_and_o1_matches_o2():
    g0 = inputs.config1(0)
    adj, colour = g0.dense()
    g, res, vm, em = run_dense(adj, colour, 4)
    cnt, vin, ein = g.kcliques()
    assert cnt > 0
    assert np.all(vm >= vin)
    rp, ci = inputs.dense_to_csr(adj)
    em_csr = em[np.repeat(np.arange(adj.shape[0]), np.diff(rp)), ci]
    assert np.all(em_csr >= ein)
    for seed in range(20):
        g.reset()
        g.fixpoint_random_order(seed * 7919 + 1)
        vm2, em2 = g.masks()
        assert np.array_equal(vm, vm2) and np.array_equal(em, em2)


# --------------------------------------------- the order-free definition
@pytest.mark.parametrize("seed", range(24))
def test_fixpoint_equals_greatest_stable_subgraph(seed):
    rng = np.random.default_rng(seed)
    k = int(rng.integers(2, 5))
    n = int(rng.integers(k, 9))
    colour = np.concatenate([np.arange(k), rng.integers(0, k, n - k)]).astype(np.int32)
    rng.shuffle(colour)
    pairs = [(u, v) for u in range(n) for v in range(u + 1, n) if colour[u] != colour[v]]
    rng.shuffle(pairs)
    edges = [e for e in pairs if rng.random() < 0.6][:12]
    adj = dense_from_edges(n, edges)
    g, res, vm, em = run_dense(adj, colour, k)
    V, E = setref.greatest_stable(n, edges, colour, k)
    assert set(np.nonzero(vm)[0].tolist()) == V
    assert {frozenset(e) for e in edges_of(em)} == E
    Vs, Es, rounds = setref.sync_rounds(n, edges, colour, k)
    assert Vs == V and Es == E and rounds == res["rounds"]
    g.reset()
    g.fixpoint_random_order(seed)
    vm2, em2 = g.masks()
    assert np.array_equal(vm, vm2) and np.array_equal(em, em2)


@pytest.mark.parametrize("seed", range(10))
def test_sync_rounds_match_python_reference(seed):
    rng = np.random.default_rng(100 + seed)
    k = int(rng.integers(3, 7))
    adj, colour = random_small(int(rng.integers(3, 8)), k, float(rng.uniform(0.3, 0.8)), seed)
    n = adj.shape[0]
    g, res, vm, em = run_dense(adj, colour, k)
    Vs, Es, rounds = setref.sync_rounds(n, edges_of(adj), colour, k)
    assert rounds == res["rounds"]
    assert set(np.nonzero(vm)[0].tolist()) == Vs
    assert {frozenset(e) for e in edges_of(em)} == Es


# ------------------------------------------------------------- invariants
def random_mid(seed, k=6, s=10, p=0.45):
    return random_small(s, k, p, seed)


@pytest.mark.parametrize("seed", range(6))
def test_stability_idempotence_monotonicity(seed):
    k = 5
    adj, colour = random_mid(seed, k=k)
    n = adj.shape[0]
    g, res, vm, em = run_dense(adj, colour, k)
    # I1: every survivor passes its test in the kernel
    us, ws = np.nonzero(np.triu(em, 1))
    vf, ef = g.failing(vs=np.nonzero(vm)[0], us=us, ws=ws)
    assert not vf.any() and not ef.any()
    # I2: kernelizing the kernel removes nothing (isolated dead vertices aside)
    g2, res2, vm2, em2 = run_dense(em, colour, k)
    assert np.array_equal(em2, em)
    assert np.array_equal(vm2 & vm, vm)
    # I5: deleting edges never grows the kernel
    rng = np.random.default_rng(seed)
    sub = adj.copy()
    for u, v in edges_of(adj):
        if rng.random() < 0.1:
            sub[u, v] = sub[v, u] = 0
    g3, res3, vm3, em3 = run_dense(sub, colour, k)
    assert np.all(em3 <= em) and np.all(vm3 <= vm)


def exact_worklist_tests(adj, colour, k):
    """Edge tests on exact worklists, from the Python set reference."""
    n = adj.shape[0]
    V = set(range(n))
    E = {frozenset(e) for e in edges_of(adj)}
    tests = len(E)
    while True:
        nb = setref._adj(n, [tuple(e) for e in E])
        fv = {v for v in V if setref.colour_index_vertex(nb, colour, v) < k - 1}
        fe = {e for e in E if setref.colour_index_edge(nb, colour, *tuple(e)) < k - 2}
        if not fv and not fe:
            return tests
        gone = {e for e in E if e in fe or (e & fv)}
        touched = set().union(*gone) if gone else set()
        V -= fv
        E -= gone
        tests += sum(1 for e in E if e & touched)


@pytest.mark.parametrize("seed", range(6))
def test_edge_test_count(seed):
    k = 4
    adj, colour = random_small(8, k, 0.35 + 0.05 * seed, seed)
    g, res, vm, em = run_dense(adj, colour, k)
    assert res["edge_tests"] == exact_worklist_tests(adj, colour, k)


# --------------------------------------------------------- formats
@pytest.mark.parametrize("seed", range(4))
def test_formats_agree(seed):
    gr = inputs.make_graph([7, 12, 5, 9, 3], 0.5, seed=seed, gid=3, plant=True)
    k = 5
    adj, colour = gr.dense()
    rd = kernelize_dense(adj, colour, k)
    rows, scol, lay = gr.bitset()
    rb = kernelize_bitset(rows, scol, k)
    rp, ci = inputs.dense_to_csr(adj)
    rc = kernelize_csr(rp, ci, colour, k)
    for key in ("rounds", "surv_vertices", "surv_edges", "edge_tests"):
        assert rd[key] == rb[key] == rc[key]
    # dense (caller order) -> slot order
    o = gr.order
    slot_adj = np.zeros_like(rd["emask"])
    slot_adj[np.ix_(o, o)] = rd["emask"]
    assert np.array_equal(inputs.unpack_rows(rb["emask"], lay).astype(np.uint8), slot_adj)
    vm_slot = np.zeros_like(rd["vmask"])
    vm_slot[o] = rd["vmask"]
    assert np.array_equal(rb["vmask"], vm_slot)
    em_csr = rd["emask"][np.repeat(np.arange(adj.shape[0]), np.diff(rp)), ci]
    assert np.array_equal(rc["emask"], em_csr)


# --------------------------------------------------------- validation
def test_validation_statuses():
    colour = np.array([0, 1, 2, 0], np.int32)
    good = dense_from_edges(4, [(0, 1), (1, 2), (2, 3)])
    assert kernelize_dense(good, colour, 3)["status"] == 0
    assert kernelize_dense(good, np.array([0, 1, 3, 0], np.int32), 3)["status"] == -2
    bad = good.copy(); bad[0, 3] = bad[3, 0] = 1            # same class
    assert kernelize_dense(bad, colour, 3)["status"] == -3
    bad = good.copy(); bad[0, 2] = 1                         # one direction
    assert kernelize_dense(bad, colour, 3)["status"] == -4
    bad = good.copy(); bad[1, 1] = 1
    assert kernelize_dense(bad, colour, 3)["status"] == -5
    bad = good.copy(); bad[0, 1] = 2
    assert kernelize_dense(bad, colour, 3)["status"] == -1
    # priority: malformed > self-loop > asymmetric > intra-class; colours first of all
    bad = good.copy(); bad[1, 1] = 1; bad[0, 2] = 1; bad[0, 3] = bad[3, 0] = 1
    assert kernelize_dense(bad, colour, 3)["status"] == -5
    bad[2, 2] = 7
    assert kernelize_dense(bad, colour, 3)["status"] == -1
    assert kernelize_dense(bad, np.array([0, 1, 5, 0], np.int32), 3)["status"] == -2
    with pytest.raises(OracleError):
        OracleGraph(FMT_DENSE, 4, 0, colour, adj=good)


def test_validation_bitset_and_csr():
    gr = inputs.make_graph([3, 4, 2], 0.7, seed=1, gid=0, shuffle=False)
    rows, col, lay = gr.bitset()
    assert kernelize_bitset(rows, col, 3)["status"] == 0
    assert kernelize_bitset(rows, col[::-1].copy(), 3)["status"] == -1          # not class-major
    assert kernelize_bitset(rows[:, :-1], col, 3)["status"] == -1               # wrong stride
    bad = rows.copy(); bad[0, 0] |= np.uint64(1 << 5)                              # padding bit
    assert kernelize_bitset(bad, col, 3)["status"] == -1
    bad = rows.copy(); bad[0, 0] |= np.uint64(1)                                   # self-loop
    assert kernelize_bitset(bad, col, 3)["status"] == -5
    bad = rows.copy(); bad[0, 0] |= np.uint64(2); bad[1, 0] |= np.uint64(1)        # intra-class pair
    assert kernelize_bitset(bad, col, 3)["status"] == -3
    adj, colour = gr.dense()
    rp, ci = inputs.dense_to_csr(adj)
    assert kernelize_csr(rp, ci, colour, 3)["status"] == 0
    if ci.size >= 2 and rp[1] - rp[0] >= 2:
        bad = ci.copy(); bad[0], bad[1] = bad[1], bad[0]
        assert kernelize_csr(rp, bad, colour, 3)["status"] == -1
    bad_rp = rp.copy(); bad_rp[-1] += 1
    assert kernelize_csr(bad_rp, ci, colour, 3)["status"] == -1


# ----------------------------------------- per-element failure report (failing)
def test_failing_reports_the_figure8_edges_that_fail():
    """Thesis section 4.2: the edge index of {a,d} is 0 and of {h,i} is 1, both
    below k-2 = 2 at k = 4; on the completion {f,h} has the single common
    neighbour i (index 1) and fails too, and so does every other edge (the
    hand derivation removes all nine in round 1)."""
    fx, idx, colour, adj = load_fig8()
    g = OracleGraph(FMT_DENSE, len(idx), fx["k"], colour, adj=adj)
    names = [("a", "d"), ("f", "h"), ("h", "i")]
    us = np.array([idx[a] for a, _ in names])
    ws = np.array([idx[b] for _, b in names])
    _, ef = g.failing(us=us, ws=ws)
    assert ef.tolist() == [1, 1, 1]
    eu, ev = np.nonzero(np.triu(adj, 1))
    _, ef = g.failing(us=eu, ws=ev)
    assert ef.all() and ef.size == 9
    # a pair that is not an edge never "fails"
    _, ef = g.failing(us=np.array([idx["a"]]), ws=np.array([idx["e"]]))
    assert ef.tolist() == [0]


@pytest.mark.parametrize("k,s", [(3, 2), (4, 3), (5, 2)])
def test_failing_reports_no_edge_of_a_complete_multipartite_graph(k, s):
    colour = np.repeat(np.arange(k), s).astype(np.int32)
    adj = (colour[:, None] != colour[None, :]).astype(np.uint8)
    g = OracleGraph(FMT_DENSE, adj.shape[0], k, colour, adj=adj)
    eu, ev = np.nonzero(np.triu(adj, 1))
    vf, ef = g.failing(vs=np.arange(adj.shape[0]), us=eu, ws=ev)
    assert ef.size == len(eu) and not ef.any() and not vf.any()
    # drop one class entirely: every edge then lacks a common neighbour there
    # (k >= 3), and every vertex outside it lacks a neighbour there
    keep = colour != k - 1
    sub = adj * keep[:, None] * keep[None, :]
    g2 = OracleGraph(FMT_DENSE, adj.shape[0], k, colour, adj=sub.astype(np.uint8))
    eu, ev = np.nonzero(np.triu(sub, 1))
    vf, ef = g2.failing(vs=np.nonzero(keep)[0], us=eu, ws=ev)
    assert ef.all() and vf.all()


# ----------------------------------------- installing a state (set_masks)
@pytest.mark.parametrize("seed", range(3))
def test_set_masks_round_trips_in_every_format_and_resumes(seed):
    """A state installed with set_masks reads back unchanged, and resuming
    from the kernel removes nothing (the kernel is a fixpoint, invariant I2)."""
    gr = inputs.make_graph([6, 9, 4, 7], 0.5, seed=seed, gid=5, plant=True)
    k = 4
    adj, colour = gr.dense()
    rows, scol, lay = gr.bitset()
    rp, ci = inputs.dense_to_csr(adj)
    makers = {
        "dense": lambda: OracleGraph(FMT_DENSE, adj.shape[0], k, colour, adj=adj),
        "bitset": lambda: OracleGraph(FMT_BITSET, rows.shape[0], k, scol, rows=rows, row_words=rows.shape[1]),
        "csr": lambda: OracleGraph(FMT_CSR, adj.shape[0], k, colour, row_ptr=rp, col_idx=ci),
    }
    for name, make in makers.items():
        ref = make()
        r = ref.fixpoint()
        vm, em = ref.masks()
        g = make()
        assert g.set_masks(vm, em), name
        vm2, em2 = g.masks()
        assert np.array_equal(vm, vm2) and np.array_equal(em, em2), name
        r2 = g.fixpoint()
        assert r2["rounds"] == 0 and r2["surv_edges"] == r["surv_edges"], name
        assert r2["surv_vertices"] == r["surv_vertices"], name
        # installing the input itself resumes to the same kernel and rounds
        g3 = make()
        vin, ein = g3.masks()
        assert g3.set_masks(vin, ein)
        assert g3.fixpoint() == r, name


def test_set_masks_rejects_states_that_are_not_subgraphs():
    gr = inputs.make_graph([5, 5, 5], 0.6, seed=2, gid=1)
    adj, colour = gr.dense()
    n = adj.shape[0]
    g = OracleGraph(FMT_DENSE, n, 3, colour, adj=adj)
    vm = np.ones(n, np.uint8)
    u, v = edges_of(adj)[0]
    one_way = adj.copy(); one_way[u, v] = 0          # alive in one direction only
    assert not g.set_masks(vm, one_way)
    dead = vm.copy(); dead[u] = 0                    # alive edge at a dead vertex
    assert not g.set_masks(dead, adj)
    extra = adj.copy()
    a, b = np.nonzero((adj == 0) & (colour[:, None] != colour[None, :]) & ~np.eye(n, dtype=bool))
    extra[a[0], b[0]] = extra[b[0], a[0]] = 1        # an edge the input does not have
    assert not g.set_masks(vm, extra)
    bad = vm.copy(); bad[0] = 2
    assert not g.set_masks(bad, adj)
    assert g.set_masks(vm, adj)


# ------------------------------------------- O3: the rounds on plain bit rows
from oracle import fixpoint_rows  # noqa: E402


def to_rows(adj, colour, k):
    """Dense (any vertex order) -> class-major bit rows with sorted colours."""
    order = np.argsort(colour, kind="stable")
    sizes = np.bincount(colour, minlength=k)
    lay = inputs.class_layout(sizes)
    slot = adj[np.ix_(order, order)].astype(bool)
    return inputs.pack_rows(slot, lay), np.sort(colour).astype(np.int32), order, lay


def same_as_o1(rows, col, k):
    a = fixpoint_rows(rows, col, k)
    b = kernelize_bitset(rows, col, k)
    assert a["status"] == b["status"]
    if a["status"]:
        return a
    for key in ("rounds", "equals_input", "surv_vertices", "surv_edges", "edge_tests"):
        assert a[key] == b[key], key
    assert np.array_equal(a["vmask"], b["vmask"]) and np.array_equal(a["emask"], b["emask"])
    return a


@pytest.mark.parametrize("seed", range(10))
def test_o3_equals_o1_on_seeded_graphs(seed):
    rng = np.random.default_rng(seed)
    k = int(rng.integers(1, 8))
    sizes = rng.integers(0 if seed % 3 == 0 else 1, 140, size=k)     # ragged, some empty classes
    p = float(rng.uniform(0.15, 0.85))
    g = inputs.make_graph(sizes, p, seed=seed, gid=9, plant=bool(sizes.min() > 0 and seed % 2), shuffle=False)
    rows, col, lay = g.bitset()
    same_as_o1(rows, col, k)


def test_o3_figure8_fixpoint_hand_derived():
    fx, idx, colour, adj = load_fig8()
    rows, col, order, lay = to_rows(adj, colour, fx["k"])
    r = same_as_o1(rows, col, fx["k"])
    assert r["rounds"] == fx["expected_fixpoint"]["rounds"] == 2
    assert r["surv_vertices"] == 0 and r["surv_edges"] == 0


@pytest.mark.parametrize("seed,p", [(0, 0.3), (1, 0.5), (2, 0.7)])
def test_o3_k3_kernel_is_union_of_triangles(seed, p):
    adj, colour = random_small(9, 3, p, seed)
    rows, col, order, lay = to_rows(adj, colour, 3)
    r = fixpoint_rows(rows, col, 3)
    slot = adj[np.ix_(order, order)]
    n = slot.shape[0]
    tri = np.zeros_like(slot)
    for a, b, c in itertools.combinations(range(n), 3):
        if slot[a, b] and slot[b, c] and slot[a, c]:
            for x, y in ((a, b), (b, c), (a, c)):
                tri[x, y] = tri[y, x] = 1
    got = inputs.unpack_rows(r["emask"], lay).astype(np.uint8)
    assert np.array_equal(got, tri)
    assert np.array_equal(r["vmask"], tri.any(axis=1).astype(np.uint8))


@pytest.mark.parametrize("k,s", [(2, 3), (4, 3), (6, 1)])
def test_o3_complete_multipartite_and_index_inequality(k, s):
    colour = np.repeat(np.arange(k), s).astype(np.int32)
    adj = (colour[:, None] != colour[None, :]).astype(np.uint8)
    rows, col, _, _ = to_rows(adj, colour, k)
    r = same_as_o1(rows, col, k)
    assert r["rounds"] == 0 and r["surv_edges"] == len(edges_of(adj))
    if k >= 4:
        adj, colour = index_inequality(k)
        rows, col, _, _ = to_rows(adj, colour, k)
        r = same_as_o1(rows, col, k)
        assert r["rounds"] == 0 and r["surv_edges"] == len(edges_of(adj))


def test_o3_validation_matches_o1():
    gr = inputs.make_graph([3, 4, 2], 0.7, seed=1, gid=0, shuffle=False)
    rows, col, lay = gr.bitset()
    cases = [(rows, col), (rows, col[::-1].copy()), (rows, np.array([0, 0, 0, 1, 1, 1, 1, 2, 5], np.int32))]
    for mut in ((0, 0, 1 << 5), (0, 0, 1), (0, 0, 2), (3, 0, 1 << 1)):
        bad = rows.copy()
        bad[mut[0], mut[1]] |= np.uint64(mut[2])
        cases.append((bad, col))
    bad = rows.copy(); bad[0, 0] |= np.uint64(2); bad[1, 0] |= np.uint64(1)
    cases.append((bad, col))
    for r, c in cases:
        a, b = fixpoint_rows(r, c, 3), kernelize_bitset(r, c, 3)
        assert a["status"] == b["status"], (a["status"], b["status"])
    assert {fixpoint_rows(r, c, 3)["status"] for r, c in cases} >= {0, -1, -2, -3, -4, -5}


@pytest.mark.parametrize("k", [2, 3, 4, 6])
def test_o3_empty_class_empties_the_graph_in_one_round(k):
    colour = np.repeat(np.arange(k - 1), 3).astype(np.int32)   # class k-1 is empty
    adj = (colour[:, None] != colour[None, :]).astype(np.uint8)
    rows, col, _, _ = to_rows(adj, colour, k)
    r = same_as_o1(rows, col, k)
    assert r["rounds"] == 1 and r["surv_vertices"] == 0 and r["surv_edges"] == 0


# ------------------------------------- witness-search work (a measurement)
from oracle import witness_words  # noqa: E402


def python_witness_words(rows, col, k):
    lay = inputs.class_layout(np.bincount(col, minlength=k))
    slot = inputs.unpack_rows(rows, lay)
    words = pairs = nowit = 0
    n = slot.shape[0]
    for u in range(n):
        for v in range(u + 1, n):
            if not slot[u, v]:
                continue
            for c in range(k):
                if c in (col[u], col[v]):
                    continue
                W = int(lay.words[c])
                found = None
                for w in range(W):
                    lo = int(lay.offsets[c]) + 64 * w
                    hi = min(lo + 64, int(lay.offsets[c + 1]))
                    if np.any(slot[u, lo:hi] & slot[v, lo:hi]):
                        found = w
                        break
                words += W if found is None else found + 1
                nowit += found is None
                pairs += 1
    return {"words": words, "pairs": pairs, "no_witness": nowit}


@pytest.mark.parametrize("seed", range(4))
def test_witness_words_matches_a_python_count(seed):
    rng = np.random.default_rng(seed)
    k = int(rng.integers(3, 6))
    sizes = rng.integers(1, 150, size=k)
    g = inputs.make_graph(sizes, float(rng.uniform(0.05, 0.3)), seed=seed, gid=4, shuffle=False)
    rows, col, lay = g.bitset()
    assert witness_words(rows, col, k) == python_witness_words(rows, col, k)


def test_witness_words_closed_forms():
    # complete multipartite: every pair has a witness in the first word
    k, s = 4, 70
    colour = np.repeat(np.arange(k), s).astype(np.int32)
    adj = (colour[:, None] != colour[None, :]).astype(np.uint8)
    rows, col, _, lay = to_rows(adj, colour, k)
    m = len(edges_of(adj))
    assert witness_words(rows, col, k) == {"words": m * (k - 2), "pairs": m * (k - 2), "no_witness": 0}
    # only the second word of class 3 (slots 64..69) touches classes 0..2: the
    # pairs of an edge inside classes 0..2 with class 3 read both words
    adj2 = adj.copy()
    c3 = np.nonzero(colour == 3)[0]
    adj2[np.ix_(c3[:64], np.arange(adj.shape[0]))] = 0
    adj2[np.ix_(np.arange(adj.shape[0]), c3[:64])] = 0
    rows, col, _, lay = to_rows(adj2, colour, k)
    r = witness_words(rows, col, k)
    inner = 3 * s * s                      # edges among classes 0..2
    outer = len(edges_of(adj2)) - inner    # edges with an endpoint in class 3
    assert r["pairs"] == inner * 2 + outer * 2
    assert r["words"] == inner * (1 + 2) + outer * 2 and r["no_witness"] == 0


# ------------------------------------ more colours than the clique size (O3)
def test_o3_more_colours_hand_case():
    # classes 0..3; a triangle on classes 0, 1, 2 and a class-3 vertex joined
    # to two triangle vertices: with clique size 3 the triangle survives and
    # the class-3 vertex (two neighbour classes, no common neighbour for its
    # edges) goes with its edges; with clique size 4 (= classes) nothing has
    # a neighbour in every other class
    adj = dense_from_edges(4, [(0, 1), (1, 2), (0, 2), (3, 0), (3, 1)])
    colour = np.array([0, 1, 2, 3], np.int32)
    rows, col, order, lay = to_rows(adj, colour, 4)
    r3 = fixpoint_rows(rows, col, 4, clique=3)
    got = inputs.unpack_rows(r3["emask"], lay).astype(np.uint8)
    # the edges {3,0} and {3,1} have the common neighbour 1 / 0 in a third
    # class, so they pass too: the whole graph is made of triangles
    assert edges_of(got) == edges_of(adj) and r3["vmask"].all() and r3["rounds"] == 0
    r4 = fixpoint_rows(rows, col, 4, clique=4)
    assert r4["surv_edges"] == 0 and r4["surv_vertices"] == 0
    adj2 = dense_from_edges(4, [(0, 1), (1, 2), (0, 2), (3, 0)])
    rows2, col2, _, lay2 = to_rows(adj2, colour, 4)
    r = fixpoint_rows(rows2, col2, 4, clique=3)
    assert set(edges_of(inputs.unpack_rows(r["emask"], lay2).astype(np.uint8))) == {(0, 1), (1, 2), (0, 2)}
    assert r["vmask"].tolist() == [1, 1, 1, 0] and r["rounds"] == 1


def m_coloured(rng, m, s, p):
    sizes = rng.integers(1, s + 1, size=m)
    colour = np.repeat(np.arange(m), sizes).astype(np.int32)
    n = colour.size
    a = (rng.random((n, n)) < p).astype(np.uint8)
    a = np.triu(a, 1)
    a = a + a.T
    a[colour[:, None] == colour[None, :]] = 0
    return a, colour


@pytest.mark.parametrize("seed", range(4))
def test_o3_clique3_on_more_colours_is_union_of_triangles(seed):
    rng = np.random.default_rng(40 + seed)
    for _ in range(10):
        m = int(rng.integers(3, 7))
        adj, colour = m_coloured(rng, m, 4, float(rng.uniform(0.2, 0.7)))
        rows, col, order, lay = to_rows(adj, colour, m)
        r = fixpoint_rows(rows, col, m, clique=3)
        slot = adj[np.ix_(order, order)]
        n = slot.shape[0]
        tri = np.zeros_like(slot)
        for a, b, c in itertools.combinations(range(n), 3):
            if slot[a, b] and slot[b, c] and slot[a, c]:
                for x, y in ((a, b), (b, c), (a, c)):
                    tri[x, y] = tri[y, x] = 1
        assert np.array_equal(inputs.unpack_rows(r["emask"], lay).astype(np.uint8), tri)
        assert np.array_equal(r["vmask"], tri.any(axis=1).astype(np.uint8))
        # clique size 2: only isolated vertices go, every edge stays
        r2 = fixpoint_rows(rows, col, m, clique=2)
        assert np.array_equal(inputs.unpack_rows(r2["emask"], lay).astype(np.uint8), slot)
        assert np.array_equal(r2["vmask"], slot.any(axis=1).astype(np.uint8))


@pytest.mark.parametrize("seed", range(4))
def test_o3_more_colours_soundness_and_monotonicity(seed):
    rng = np.random.default_rng(60 + seed)
    for _ in range(8):
        m = int(rng.integers(3, 7))
        adj, colour = m_coloured(rng, m, 3, float(rng.uniform(0.4, 0.9)))
        rows, col, order, lay = to_rows(adj, colour, m)
        slot = adj[np.ix_(order, order)]
        prev = None
        for kk in range(1, m + 1):
            r = fixpoint_rows(rows, col, m, clique=kk)
            got = inputs.unpack_rows(r["emask"], lay)
            # every vertex and edge of every kk-clique survives (brute force)
            for cl in itertools.combinations(range(slot.shape[0]), kk):
                if len({int(col[v]) for v in cl}) == kk and all(slot[x, y] for x, y in itertools.combinations(cl, 2)):
                    assert all(r["vmask"][v] for v in cl)
                    assert all(got[x, y] for x, y in itertools.combinations(cl, 2))
            if prev is not None:        # a larger clique size prunes at least as much
                assert not (r["vmask"] & ~prev[0]).any() and not (got & ~prev[1]).any()
            prev = (r["vmask"], got)
        # a complete m-partite graph keeps everything for every clique size
        full = (colour[:, None] != colour[None, :]).astype(np.uint8)
        rf, cf, _, _ = to_rows(full, colour, m)
        for kk in range(1, m + 1):
            assert fixpoint_rows(rf, cf, m, clique=kk)["rounds"] == 0
