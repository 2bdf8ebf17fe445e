"""Struction on the GPU (kz_struction, through the C ABI) against the oracle
(Definition 4.1.1 as read in oracle/kz_oracle_ext.c, pinned by Theorem 1):
the node map and every adjacency bit of G' are equal, on random graphs and
pivots, word-boundary sizes, pivots adjacent to all or to none, and the
input errors."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import struction  # noqa: E402
from paper_2212_00574_amd import inputs  # noqa: E402
from paper_2212_00574_amd.binding import Kernelizer  # noqa: E402

DEV = torch.device("cuda", 0)


@pytest.fixture(scope="module")
def kz():
    k = Kernelizer(0)
    yield k
    k.close()


def random_graph(rng, n, p):
    a = (rng.random((n, n)) < p).astype(np.uint8)
    a = np.triu(a, 1)
    return a + a.T


def check(kz, adj, pivot, ctx):
    ref, rmap = struction(adj, pivot)
    rows = torch.from_numpy(inputs.dense_to_rows(adj).view(np.int64)).to(DEV)
    out, mp, res = kz.struction(rows, pivot)
    torch.cuda.synchronize()
    npr = ref.shape[0]
    assert res["status"] == 0 and res["nodes"] == npr, (ctx, res, npr)
    assert res["a_nodes"] == int(adj[pivot].sum()) and res["input_edges"] == int(adj.sum()) // 2, ctx
    if npr == 0:
        return
    assert np.array_equal(mp.cpu().numpy(), rmap), ctx
    got = inputs.rows_to_dense(out.cpu().numpy(), npr)
    assert np.array_equal(got, ref), ctx


@pytest.mark.parametrize("seed", range(3))
def test_random_graphs_match_oracle(kz, seed):
    rng = np.random.default_rng(900 + seed)
    for i in range(30):
        n = int(rng.integers(1, 160))
        adj = random_graph(rng, n, float(rng.uniform(0.02, 0.6)))
        check(kz, adj, int(rng.integers(0, n)), (seed, i, n))


def test_word_boundaries_and_pivots(kz):
    rng = np.random.default_rng(3)
    for n in (63, 64, 65, 129):
        adj = random_graph(rng, n, 0.2)
        for pivot in (0, n // 2, n - 1):
            check(kz, adj, pivot, (n, pivot))
    star = np.zeros((70, 70), np.uint8)
    star[0, 1:] = star[1:, 0] = 1
    check(kz, star, 0, "pivot adjacent to all: G' = G[A]")
    check(kz, star, 5, "pivot of degree one")
    check(kz, np.zeros((5, 5), np.uint8), 2, "edgeless")
    check(kz, np.zeros((1, 1), np.uint8), 0, "one vertex: G' is empty")


def test_thesis_sized_graph(kz):
    # 600 vertices at p = 0.1: about 60 A nodes and 15 000 C nodes
    adj = random_graph(np.random.default_rng(11), 600, 0.1)
    check(kz, adj, 0, "n = 600")


def test_statuses(kz):
    rng = np.random.default_rng(4)
    adj = random_graph(rng, 80, 0.3)
    bad = adj.copy()
    bad[2, 60] = 1 - bad[2, 60]
    rows = torch.from_numpy(inputs.dense_to_rows(bad).view(np.int64)).to(DEV)
    _, _, res = kz.struction(rows, 0, check=False)
    assert res["status"] == -4
    loop = adj.copy()
    loop[9, 9] = 1
    rows = torch.from_numpy(inputs.dense_to_rows(loop).view(np.int64)).to(DEV)
    _, _, res = kz.struction(rows, 0, check=False)
    assert res["status"] == -5
    rows = torch.from_numpy(inputs.dense_to_rows(adj).view(np.int64)).to(DEV)
    _, _, res = kz.struction(rows, 80, check=False)
    assert res["status"] == -1
