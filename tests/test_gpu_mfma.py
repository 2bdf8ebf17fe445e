"""The int8 MFMA count path of the edge test against the oracle (bit-exact),
and against the witness-search path at the full dense workload: the same
masks, rounds and counts are required."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import kernelize_bitset, kernelize_dense  # noqa: E402
from paper_2212_00574_amd import inputs  # noqa: E402
from paper_2212_00574_amd.binding import KZ_EDGE_BITSET, KZ_EDGE_MFMA_I8, Kernelizer, KzError  # noqa: E402

from test_gpu_parity import CASES, check_same, run_bitset, run_dense  # noqa: E402

DEV = torch.device("cuda", 0)


@pytest.fixture(scope="module")
def kzm():
    k = Kernelizer(0)
    k.set_edge_path(KZ_EDGE_MFMA_I8)
    yield k
    k.close()


def both(kzm, g, k, ctx):
    adj, colour = g.dense()
    res, vm, em = run_dense(kzm, adj, colour, k, ctx + " mfma")
    check_same(res, kernelize_dense(adj, colour, k), vm, em, ctx + " dense mfma")
    rows, scol, lay = g.bitset()
    resb, vmb, emb = run_bitset(kzm, rows, scol, k, ctx + " mfma")
    ref = kernelize_bitset(rows, scol, k)
    check_same(resb, ref, vmb, emb, ctx + " bitset mfma")
    return ref


@pytest.mark.parametrize("ci", range(len(CASES)))
@pytest.mark.parametrize("seed", [0, 1])
def test_mfma_random_graphs(kzm, ci, seed):
    sizes, p, plant = CASES[ci]
    g = inputs.make_graph(sizes, p, seed=seed, gid=ci, plant=plant)
    both(kzm, g, len(sizes), "case%d/seed%d" % (ci, seed))


def test_mfma_cascades(kzm):
    seen = []
    for seed in range(8):
        g = inputs.make_graph([60] * 6, 0.16, seed=seed, gid=99)
        seen.append(both(kzm, g, 6, "cascade/seed%d" % seed)["rounds"])
    g = inputs.make_graph([130, 129, 128, 127, 200], 0.12, seed=3, gid=5)   # group tiles with ragged blocks
    seen.append(both(kzm, g, 5, "ragged")["rounds"])
    assert max(seen) >= 3, seen


def test_mfma_config3a_equals_bitset_path(kzm):
    """The dense workload (k=20 x 1000, p=0.3): both edge-test paths agree."""
    g = inputs.config3a(0)
    rows, col, lay = g.bitset()
    t_rows = torch.from_numpy(rows.view(np.int64)).to(DEV)
    t_col = torch.from_numpy(col).to(DEV)
    vm1, em1, r1 = kzm.kernelize_bitset(t_rows, t_col, 20)
    ref = Kernelizer(0)
    ref.set_edge_path(KZ_EDGE_BITSET)
    vm2, em2, r2 = ref.kernelize_bitset(t_rows, t_col, 20)
    torch.cuda.synchronize()
    assert r1 == r2
    assert torch.equal(vm1, vm2) and torch.equal(em1, em2)
    ref.close()


def test_mfma_row_limit(kzm):
    """Rows of more than 2048 words are beyond the MFMA path: the call is
    refused with KZ_ETOOLARGE before anything is launched."""
    from paper_2212_00574_amd.binding import KZ_ETOOLARGE
    k = n = 2049                            # one vertex per class: 2049 words per row
    rows = torch.zeros((n, k), dtype=torch.int64, device=DEV)
    col = torch.arange(n, dtype=torch.int32, device=DEV)
    with pytest.raises(KzError) as err:
        kzm.kernelize_bitset(rows, col, k)
    assert err.value.status == KZ_ETOOLARGE


def test_edge_path_argument(kzm):
    with pytest.raises(KzError):
        kzm.set_edge_path(7)
