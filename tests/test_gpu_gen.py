"""The device materialiser writes exactly the bit rows the host generator
draws (same SplitMix64 edge rule, same planted clique), bit for bit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2212_00574_amd import inputs  # noqa: E402
from paper_2212_00574_amd.binding import Kernelizer, KzError, kz_gen_bitset  # noqa: E402

DEV = torch.device("cuda", 0)

CASES = [
    ([25] * 4, 0.5, 0, 0, False),
    ([70, 40, 90, 65], 0.35, 3, 7, True),
    ([1, 64, 65, 0, 128, 3], 0.8, 11, 2, False),
    ([300] * 10, 0.6, 0, 0, True),
    ([200, 17, 129, 64, 63, 5, 190], 0.1, 5, 4000000000, True),
    ([12] * 30, 0.9, 2**32 - 1, 1, False),
    ([40, 40], 0.0, 1, 1, True),
    ([33, 31, 30], 1.0, 9, 9, False),
]


@pytest.fixture(scope="module")
def kz():
    k = Kernelizer(0)
    yield k
    k.close()


@pytest.mark.parametrize("case", range(len(CASES)))
def test_device_rows_equal_host_rows(kz, case):
    sizes, p, seed, gid, plant = CASES[case]
    if plant and 0 in sizes:
        plant = False
    g = inputs.make_graph(sizes, p, seed=seed, gid=gid, plant=plant, shuffle=False)
    rows, col, lay = g.bitset()
    print("gen", sizes, p, seed, gid, plant, flush=True)
    out = torch.full((max(lay.n * lay.R, 1),), -1, dtype=torch.int64, device=DEV)
    colour = torch.full((max(lay.n, 1),), -7, dtype=torch.int32, device=DEV)
    kz_gen_bitset(kz.ctx, sizes, p, seed, gid, g.planted, out.data_ptr(), lay.R, colour.data_ptr(), None)
    torch.cuda.synchronize()
    got = out.cpu().numpy()[:lay.n * lay.R].view(np.uint64).reshape(lay.n, lay.R)
    assert np.array_equal(got, rows)
    assert np.array_equal(colour.cpu().numpy()[:lay.n], col)


def test_argument_errors(kz):
    out = torch.zeros(16, dtype=torch.int64, device=DEV)
    with pytest.raises(KzError):
        kz_gen_bitset(kz.ctx, [10, 10], 0.5, 0, 0, None, out.data_ptr(), 3, None, None)   # row_words is 2
    with pytest.raises(KzError):
        kz_gen_bitset(kz.ctx, [10, 10], 1.5, 0, 0, None, out.data_ptr(), 2, None, None)
    with pytest.raises(KzError):
        kz_gen_bitset(kz.ctx, [10, 10], 0.5, 0, 0, [3, 5], out.data_ptr(), 2, None, None)  # 5 is not in class 1
