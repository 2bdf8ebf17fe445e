"""Seeded generators: reproducible, legal, and in the documented layouts."""
import numpy as np
import pytest

from paper_2212_00574_amd import inputs


def test_splitmix64_published_vector():
    # SplitMix64 started at 1234567: the first five outputs published with the
    # reference implementation of Steele, Lea and Flood's generator.
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    s, got = 1234567, []
    for _ in range(5):
        got.append(inputs.splitmix64_int(s))
        s = (s + 0x9E3779B97F4A7C15) % 2**64
    assert got == want
    xs = np.array([1234567 + i * 0x9E3779B97F4A7C15 % 2**64 for i in range(5)], np.uint64)
    assert inputs.splitmix64(xs).tolist() == want


def test_threshold_exact():
    assert inputs.edge_threshold(0.5) == 2**63
    assert inputs.edge_threshold(0.0) == 0
    assert inputs.edge_threshold(1.0) == 2**64 - 1


def test_graph_is_legal_symmetric_and_reproducible():
    g = inputs.make_graph([5, 9, 64, 65, 1], 0.4, seed=3, gid=11, plant=True)
    adj, colour = g.dense()
    assert np.array_equal(adj, adj.T)
    assert not adj.diagonal().any()
    assert not adj[colour[:, None] == colour[None, :]].any()
    adj2, colour2 = inputs.make_graph([5, 9, 64, 65, 1], 0.4, seed=3, gid=11, plant=True).dense()
    assert np.array_equal(adj, adj2) and np.array_equal(colour, colour2)
    # planted clique: one vertex per class, pairwise adjacent (slot ids)
    slot = g.dense_slot()
    pl = g.planted
    assert len(pl) == 5
    assert all(slot[a, b] for a in pl for b in pl if a != b)
    # scalar draw agrees with the block draw
    lay = g.layout
    col = inputs.sorted_colour(g.sizes)
    for a, b in [(0, 7), (3, 100), (20, 142)]:
        if col[a] != col[b] and not ({a, b} <= set(pl.tolist())):
            assert slot[a, b] == inputs.pair_is_edge(3, 11, a, b, 0.4)
    assert lay.R == 1 + 1 + 1 + 2 + 1


def test_bitset_roundtrip_and_padding():
    g = inputs.make_graph([70, 3, 128, 64], 0.5, seed=1, gid=2, shuffle=False)
    rows, colour, lay = g.bitset(chunk=17)
    assert rows.shape == (g.n, lay.R)
    back = inputs.unpack_rows(rows, lay)
    assert np.array_equal(back.astype(np.uint8), g.dense_slot())
    # padding bits of every segment are zero
    for c in range(lay.k):
        s, w = int(lay.sizes[c]), int(lay.words[c])
        if s % 64:
            last = rows[:, lay.segoff[c] + w - 1]
            assert not np.any(last >> np.uint64(s % 64))


def test_csr_roundtrip():
    g = inputs.make_graph([4, 6, 5], 0.6, seed=2)
    adj, colour = g.dense()
    rp, ci = inputs.dense_to_csr(adj)
    assert np.array_equal(inputs.csr_to_dense(adj.shape[0], rp, ci), adj)
    for u in range(adj.shape[0]):
        assert np.all(np.diff(ci[rp[u]:rp[u + 1]]) > 0)


def test_sparse_generator():
    sg = inputs.make_sparse(2000, 7, 5000, seed=4)
    assert sg.sizes.sum() == 2000
    assert sg.row_ptr[-1] == 2 * 5000
    src = np.repeat(np.arange(sg.n), np.diff(sg.row_ptr))
    assert np.all(sg.colour[src] != sg.colour[sg.col_idx])
    key = set(zip(src.tolist(), sg.col_idx.tolist()))
    assert all((b, a) in key for a, b in key)


def test_config_specs():
    c4 = inputs.config4_specs(0, graphs=200)
    assert all(4 <= s.k <= 16 and 0.2 <= s.p <= 0.8 for s in c4)
    assert all(np.all((s.sizes >= 8) & (s.sizes <= 128)) for s in c4)
    c5 = inputs.config5_specs(0, requests=300)
    assert all(200 <= s.n <= 20000 and 5 <= s.k <= 30 for s in c5)
    assert all(s.sizes.max() - s.sizes.min() <= 1 and s.sizes.sum() == s.n for s in c5)
    t = [s.arrival_s for s in c5]
    assert all(b > a for a, b in zip(t, t[1:]))


@pytest.mark.parametrize("fn,n,k", [(inputs.config1, 100, 4)])
def test_config1_shape(fn, n, k):
    g = fn(0)
    adj, colour = g.dense()
    assert adj.shape == (n, n) and len(np.unique(colour)) == k
