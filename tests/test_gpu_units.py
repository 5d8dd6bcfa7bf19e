"""GPU units through the C ABI: the LDS radix sort, the cell-table builder and the
pass-rate reduction, each against its plain definition."""
import numpy as np
import pytest

from gpu_util import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gx():
    import paper_1012_1900_amd as g
    return g


def _i32(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to("cuda")


@pytest.mark.parametrize("n", [0, 1, 5, 255, 1313, 4096, 4097, 100003, (1 << 20) + 17])
@pytest.mark.parametrize("kind", ["random", "few_keys", "float_bits"])
def test_radix_sort_stable(gx, n, kind):
    rng = np.random.default_rng(n + len(kind))
    if kind == "random":
        keys = rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
    elif kind == "few_keys":
        keys = rng.integers(0, 7, size=n).astype(np.uint32) * np.uint32(0x01010101)
    else:
        keys = (rng.exponential(0.3, size=n) ** 2).astype(np.float32).view(np.uint32)
    vals = np.arange(n, dtype=np.uint32)
    k, v = _i32(keys), _i32(vals)
    gx.sort_pairs(k, v)
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(host(k).view(np.uint32), keys[order])
    assert np.array_equal(host(v).view(np.uint32), vals[order])


def _table_reference(shape, s, radius):
    """Every cell offset a with key(a)^2 < radius^2 (plain enumeration, FP64)."""
    nd = len(shape)
    rngs = []
    for n, si in zip(shape, s):
        c = int(np.ceil(radius / si)) + 1
        rngs.append(np.arange(max(-(n - 1), -c - 1), min(n - 1, c) + 1))
    A = np.stack([x.ravel() for x in np.meshgrid(*rngs, indexing="ij")], axis=1)
    m = np.where(A > 0, A, np.where(A < -1, -A - 1, 0)).astype(np.float64)
    key2 = np.sum((m * np.asarray(s)) ** 2, axis=1)
    keep = key2 < radius * radius
    return A[keep], key2[keep]


@pytest.mark.parametrize("shape,s,radius", [
    ((96, 128, 128), (0.8333333333333334,) * 3, 5.1),
    ((20, 30, 40), (1.5, 1.0, 0.4), 3.7),
    ((64, 64), (1.0 / 3.0, 1.0 / 3.0), 4.8),
    ((5, 6, 7), (1.0, 1.0, 1.0), 50.0),      # radius beyond the grid: the whole box
])
def test_cell_table(gx, shape, s, radius):
    key2, offs = gx.build_table(shape, s, radius)
    key2, offs = host(key2), host(offs)[:, : len(shape)]
    A, k2 = _table_reference(shape, s, radius)
    assert key2.shape[0] == A.shape[0]
    # ascending, rounded toward -inf: float(key2) <= exact < next float up
    assert np.all(np.diff(key2) >= 0)
    got = {tuple(r) for r in offs}
    assert got == {tuple(r) for r in A}
    exact = dict(zip(map(tuple, A), k2))
    ex = np.array([exact[tuple(r)] for r in offs])
    assert np.all(key2.astype(np.float64) <= ex)
    assert np.all(np.nextafter(key2, np.float32(np.inf)).astype(np.float64) > ex)
    # ties keep the enumeration order (slowest axis first, ascending)
    same = np.flatnonzero(np.diff(key2) == 0)
    for j in same[:2000]:
        assert tuple(offs[j]) < tuple(offs[j + 1])


def test_pass_count(gx):
    rng = np.random.default_rng(3)
    g = rng.uniform(-1.0, 2.0, size=100001).astype(np.float32)
    g[g < 0] = -1.0
    g[:5] = [1.0, 1.0 + 1e-6, 1.0 - 1e-6, 1.00002, 0.0]
    n_eval, n_pass, n_border = gx.pass_count(dev(g))
    assert n_eval == int(np.sum(g >= 0))
    assert n_pass == int(np.sum((g >= 0) & (g <= 1)))
    assert n_border == int(np.sum((g >= 0) & (np.abs(g - np.float32(1.0)) <= np.float32(1e-5))))
