"""Upstream legal colouring on the GPU (Jones-Plassmann, kz_colour_jp): the
colours, rounds and colour counts equal the oracle's exactly on seeded
graphs; bad input gets its status; and uncoloured graphs go end to end:
coloured on the GPU, laid out class by class, and kernelized by the batched
path with the clique size below the number of colours, equal to the
oracle's O3 on the same classes, with a planted clique surviving."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import colour_jp, fixpoint_rows  # noqa: E402
from paper_2212_00574_amd import inputs  # noqa: E402
from paper_2212_00574_amd.binding import Batch, BatchKernelizer, Kernelizer, KzError  # noqa: E402

DEV = torch.device("cuda", 0)


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def kz():
    k = Kernelizer(0)
    yield k
    k.close()


def random_graph(n, p, seed, plant=0):
    """A seeded G(n, p), plus a clique on `plant` random vertices; uint64
    priorities drawn from the same generator."""
    rng = np.random.default_rng(seed)
    a = np.triu((rng.random((n, n)) < p).astype(np.uint8), 1)
    a = a | a.T
    clique = np.sort(rng.choice(n, size=plant, replace=False)) if plant else np.zeros(0, np.int64)
    for i in clique:
        for j in clique:
            if i != j:
                a[i, j] = 1
    pri = rng.integers(0, 2**64, size=n, dtype=np.uint64)
    return a, pri, clique


def gpu_colour(kz, a, pri, row_words=None):
    rows = inputs.dense_to_rows(a)
    if row_words is not None and row_words > rows.shape[1]:
        rows = np.pad(rows, ((0, 0), (0, row_words - rows.shape[1])))
    t_rows = torch.from_numpy(rows.view(np.int64)).to(DEV)
    t_pri = torch.from_numpy(pri.view(np.int64)).to(DEV)
    col, res = kz.colour_jp(t_rows, a.shape[0], t_pri)
    torch.cuda.synchronize()
    return col.cpu().numpy(), res


CASES = [(1, 0.5, 1), (2, 1.0, 2), (63, 0.3, 3), (64, 0.5, 4), (65, 0.5, 5), (300, 0.05, 6), (500, 0.5, 7),
         (777, 0.9, 8), (1500, 0.2, 9), (4000, 0.02, 10), (3000, 0.3, 11)]


@pytest.mark.parametrize("n,p,seed", CASES)
def test_colouring_equals_oracle(kz, n, p, seed):
    a, pri, _ = random_graph(n, p, seed)
    say("colour_jp", n, p)
    col, res = gpu_colour(kz, a, pri)
    ref, rounds, nc = colour_jp(a, pri)
    assert res["status"] == 0
    assert np.array_equal(col, ref), (n, p)
    assert res["rounds"] == rounds and res["colours"] == nc
    # legal, whatever the oracle says
    u, v = np.nonzero(a)
    assert np.all(col[u] != col[v])


def test_colouring_special_graphs(kz):
    rng = np.random.default_rng(12)
    for n in (5, 130):
        full = np.ones((n, n), np.uint8) - np.eye(n, dtype=np.uint8)
        pri = rng.integers(0, 2**64, size=n, dtype=np.uint64)
        col, res = gpu_colour(kz, full, pri)
        assert sorted(col.tolist()) == list(range(n)) and res["rounds"] == n
        assert np.array_equal(col, colour_jp(full, pri)[0])
        col, res = gpu_colour(kz, np.zeros((n, n), np.uint8), pri)
        assert col.tolist() == [0] * n and res["rounds"] == 1 and res["colours"] == 1
        # equal priorities: ties broken by the index
        col, _ = gpu_colour(kz, full, np.zeros(n, np.uint64))
        assert col.tolist() == list(range(n - 1, -1, -1))
    # rows wider than needed
    a, pri, _ = random_graph(100, 0.3, 13)
    col, _ = gpu_colour(kz, a, pri, row_words=5)
    assert np.array_equal(col, colour_jp(a, pri)[0])


def test_colouring_rejects_bad_rows(kz):
    a, pri, _ = random_graph(90, 0.3, 14)
    t_pri = torch.from_numpy(pri.view(np.int64)).to(DEV)

    def status(rows):
        t = torch.from_numpy(rows.view(np.int64)).to(DEV)
        try:
            kz.colour_jp(t, 90, t_pri)
        except KzError as e:
            return e.status
        return 0

    rows = inputs.dense_to_rows(a)
    bad = rows.copy(); bad[3, 0] |= np.uint64(1 << 3)               # self-loop
    assert status(bad) == -5
    u = int(np.nonzero(a[0] == 0)[0][1])
    bad = rows.copy(); bad[0, u >> 6] |= np.uint64(1) << np.uint64(u & 63)   # one direction only
    assert status(bad) == -4
    bad = rows.copy(); bad[7, 1] |= np.uint64(1) << np.uint64(40)   # vertex 104 of 90
    assert status(bad) == -1
    assert status(rows) == 0


def class_major(a, col):
    """The graph laid out class by class (the bit-row format): rows, the
    sorted colours, and the vertex of each slot."""
    m = int(col.max()) + 1
    order = np.argsort(col, kind="stable")
    sizes = np.bincount(col, minlength=m)
    lay = inputs.class_layout(sizes)
    rows = inputs.pack_rows(a[np.ix_(order, order)].astype(bool), lay)
    return rows, col[order].astype(np.int32), order, m


def test_uncoloured_graphs_end_to_end(kz):
    """Colour on the GPU, then kernelize with the clique size below the
    colour count: equal to the oracle on the same classes, and the planted
    clique survives (every vertex and edge of a k-clique does)."""
    gs, meta = [], []
    for i, (n, p, plant) in enumerate(((400, 0.08, 6), (900, 0.05, 7), (250, 0.2, 8), (1200, 0.03, 5))):
        a, pri, clique = random_graph(n, p, 30 + i, plant=plant)
        col, res = gpu_colour(kz, a, pri)
        assert np.array_equal(col, colour_jp(a, pri)[0])
        rows, scol, order, m = class_major(a, col)
        say("end to end", n, p, "colours", m, "clique", plant)
        assert plant <= m <= 64
        gs.append((rows, scol, m, plant))
        meta.append((order, clique))
    b = Batch(gs, DEV)
    BatchKernelizer(kz).run(b)
    torch.cuda.synchronize()
    res = b.read_results()
    for i, (rows, scol, m, k) in enumerate(gs):
        ref = fixpoint_rows(rows, scol, m, clique=k)
        r = res[i]
        assert r["status"] == ref["status"] == 0
        assert r["rounds"] == ref["rounds"] and r["edge_tests"] == ref["edge_tests"]
        assert r["surviving_vertices"] == ref["surv_vertices"] and r["surviving_edges"] == ref["surv_edges"]
        vm, em = b.masks(i)
        assert np.array_equal(vm, ref["vmask"]) and np.array_equal(em, ref["emask"])
        order, clique = meta[i]
        slot = np.argsort(order)                 # slot of each original vertex
        assert all(vm[slot[v]] for v in clique)
