"""k-clique search on the GPU (kz_find_clique, through the C ABI) against the
oracle's class-order search (oracle/kz_oracle_ext.c, pinned by brute force):
the same lexicographically smallest clique, or none, on the input graph and
on its kernel (every k-clique survives kernelization, so the answer is the
same); live masks, multi-word classes, k = 1 and 2, empty classes, and bad
colourings."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import find_clique  # noqa: E402
from paper_2212_00574_amd import inputs  # noqa: E402
from paper_2212_00574_amd.binding import Kernelizer  # noqa: E402

DEV = torch.device("cuda", 0)


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def kz():
    k = Kernelizer(0)
    yield k
    k.close()


def case(sizes, p, seed, gid, plant):
    g = inputs.make_graph(sizes, p, seed=seed, gid=gid, plant=plant, shuffle=False)
    rows, colour, lay = g.bitset()
    adj = inputs.unpack_rows(rows, lay).astype(np.uint8)
    return rows, colour, lay, adj


def gpu(kz, rows, colour, k, vmask=None):
    r = torch.from_numpy(np.ascontiguousarray(rows).view(np.int64)).to(DEV)
    c = torch.from_numpy(np.ascontiguousarray(colour, np.int32)).to(DEV)
    vm = None if vmask is None else torch.from_numpy(np.ascontiguousarray(vmask, np.uint8)).to(DEV)
    cl, res = kz.find_clique(r, c, k, vm, check=False)
    torch.cuda.synchronize()
    return cl.cpu().numpy(), res


def same(kz, rows, colour, adj, k, vmask=None, ctx=None):
    ref, _ = find_clique(adj, colour, k, vmask)
    got, res = gpu(kz, rows, colour, k, vmask)
    assert res["status"] == 0, ctx
    assert res["found"] == (ref is not None), (ctx, res, ref)
    if ref is None:
        assert (got == -1).all(), ctx
    else:
        assert got.tolist() == ref.tolist(), (ctx, got, ref)
    return ref


@pytest.mark.parametrize("seed", range(3))
def test_random_graphs_match_oracle(kz, seed):
    rng = np.random.default_rng(70 + seed)
    found = 0
    say("clique search: random graphs, seed", seed)
    for i in range(60):
        k = int(rng.integers(1, 9))
        sizes = rng.integers(1, 90, size=k)
        p = float(rng.uniform(0.2, 0.9))
        rows, colour, lay, adj = case(sizes, p, 70 + seed, i, plant=bool(rng.random() < 0.4))
        vmask = (rng.random(lay.n) < 0.9).astype(np.uint8) if rng.random() < 0.3 else None
        found += same(kz, rows, colour, adj, k, vmask, (seed, i, k, p)) is not None
    assert found >= 10


def test_on_the_kernel(kz):
    """The search on kz_kernelize's output answers as on the input."""
    rng = np.random.default_rng(5)
    for i in range(30):
        k = int(rng.integers(3, 8))
        sizes = rng.integers(20, 130, size=k)
        p = float(rng.uniform(0.25, 0.75))
        rows, colour, lay, adj = case(sizes, p, 5, i, plant=bool(rng.random() < 0.5))
        r = torch.from_numpy(rows.view(np.int64)).to(DEV)
        c = torch.from_numpy(colour).to(DEV)
        vm, em, res = kz.kernelize_bitset(r, c, k)
        cl, cres = kz.find_clique(em, c, k, vm)
        torch.cuda.synchronize()
        ref, _ = find_clique(adj, colour, k)
        assert cres["found"] == (ref is not None), i
        if ref is not None:
            assert cl.cpu().numpy().tolist() == ref.tolist(), i


def test_multiword_classes_and_large_k(kz):
    rng = np.random.default_rng(8)
    for i, (k, s, p) in enumerate([(10, 300, 0.6), (12, 130, 0.7), (6, 700, 0.25), (16, 65, 0.8)]):
        rows, colour, lay, adj = case([s] * k, p, 8, i, plant=True)
        say("clique search: k=%d s=%d p=%.2f" % (k, s, p))
        assert same(kz, rows, colour, adj, k, ctx=(k, s, p)) is not None


def test_few_roots_children_shared(kz):
    """Few (class 0, class 1) roots and wide classes after them: nearly all
    the work is the roots' class-2 children, taken by waves that have no
    root of their own."""
    rng = np.random.default_rng(9)
    found = 0
    for i in range(12):
        k = int(rng.integers(4, 11))
        sizes = np.concatenate([rng.integers(1, 4, size=2), rng.integers(40, 130, size=k - 2)])
        p = float(rng.uniform(0.25, 0.5))
        rows, colour, lay, adj = case(sizes, p, 9, i, plant=bool(rng.random() < 0.3))
        vmask = (rng.random(lay.n) < 0.95).astype(np.uint8) if i % 3 == 0 else None
        say("clique search: few roots, k=%d p=%.2f" % (k, p))
        found += same(kz, rows, colour, adj, k, vmask, (i, k, p)) is not None
    assert found >= 3
    # wider searches before the first clique (the oracle extends 10^2 to
    # 3.4 * 10^4 partial cliques)
    for i, (sizes, p) in enumerate([([2, 2] + [100] * 10, 0.5), ([1, 1] + [120] * 8, 0.45),
                                    ([2, 3] + [128] * 12, 0.55), ([3, 3] + [110] * 9, 0.5)]):
        rows, colour, lay, adj = case(sizes, p, 13, i, plant=False)
        say("clique search: few roots, wide, k=%d p=%.2f" % (len(sizes), p))
        assert same(kz, rows, colour, adj, len(sizes), ctx=(sizes, p)) is not None


def test_stack_in_global_memory(kz):
    """k * R above the LDS stack (1024 words per wave): the stack lives in
    the workspace."""
    for i, (k, s, p, plant) in enumerate([(8, 1100, 0.3, True), (24, 65, 0.35, False), (24, 65, 0.9, True)]):
        rows, colour, lay, adj = case([s] * k, p, 11, i, plant=plant)
        assert k * lay.R > 1024
        say("clique search: global stack, k=%d s=%d p=%.2f" % (k, s, p))
        ref = same(kz, rows, colour, adj, k, ctx=(k, s, p))
        assert ref is not None or not plant


def test_degenerate_and_errors(kz):
    rows, colour, lay, adj = case([5, 0, 4], 0.9, 3, 0, plant=False)
    assert same(kz, rows, colour, adj, 3) is None                # an empty class: no clique
    rows, colour, lay, adj = case([4, 3], 0.0, 3, 1, plant=False)
    assert same(kz, rows, colour, adj, 2) is None                # no edge
    _, res = gpu(kz, rows, colour, 1)                            # colour 1 is outside [0, 1)
    assert res["status"] == -2
    rows1, colour1, lay1, adj1 = case([4], 0.0, 3, 3, plant=False)
    assert same(kz, rows1, colour1, adj1, 1).tolist() == [0]     # k = 1: the first live vertex
    dead = np.zeros(lay1.n, np.uint8)
    dead[2] = 1
    assert same(kz, rows1, colour1, adj1, 1, dead).tolist() == [2]
    assert same(kz, rows1, colour1, adj1, 1, np.zeros(lay1.n, np.uint8)) is None
    rows, colour, lay, adj = case([4, 3], 1.0, 3, 2, plant=False)
    assert same(kz, rows, colour, adj, 2).tolist() == [0, 4]
    # colours out of range / unsorted
    bad = colour.copy()
    bad[0] = 5
    _, res = gpu(kz, rows, bad, 2)
    assert res["status"] == -2
    bad = colour[::-1].copy()
    _, res = gpu(kz, rows, bad, 2)
    assert res["status"] == -1
    empty = torch.empty((0, 1), dtype=torch.int64, device=DEV)
    cl, res = kz.find_clique(empty, torch.empty(0, dtype=torch.int32, device=DEV), 3)
    torch.cuda.synchronize()
    assert res["status"] == 0 and res["found"] == 0 and (cl.cpu().numpy() == -1).all()
