"""Invariants and bounds that any correct gamma must obey (metamorphic pins).

* proportional criteria (k DD, k DTA) give gamma / k; for k = 2 every normalised
  coordinate scales exactly, so gamma and the visited-cell counts match bit for bit
  (the paper's observation that proportional criteria leave the run time unchanged,
  Sec. 3.6, is this identity of the walks);
* axis permutation (spacing permuted with it) and central inversion map the Kuhn
  triangulation onto itself;
* extrusion: a 3D pair constant along z gives the 2D gamma of each slice;
* 0 <= gamma <= gamma0; gamma is non-increasing in DD and in DTA;
* work law (Sec. 3.4): every cell with key < gamma is visited and no cell with
  key >= gamma0 is.
"""
import itertools

import numpy as np
import pytest

import oracle
from dosegen import make_pair_2d, make_pair_3d


@pytest.fixture(scope="module")
def pair3():
    return make_pair_3d(11, shape=(12, 14, 16), spacing=(2.5, 2.0, 1.5))


@pytest.fixture(scope="module")
def pair2():
    return make_pair_2d(12, shape=(40, 36), spacing=(1.0, 1.2))


def test_proportional_criteria_exact(pair3):
    p = pair3
    a = oracle.gamma(p.ref, p.eval, p.spacing, 0.03, 3.0, 0.1)
    b = oracle.gamma(p.ref, p.eval, p.spacing, 0.06, 6.0, 0.1)
    m = a.gamma >= 0
    assert np.array_equal(a.gamma[m] / 2.0, b.gamma[m])
    assert np.array_equal(a.cells, b.cells)


def test_proportional_criteria_k3(pair2):
    p = pair2
    a = oracle.gamma(p.ref, p.eval, p.spacing, 0.01, 1.0, 0.1)
    b = oracle.gamma(p.ref, p.eval, p.spacing, 0.03, 3.0, 0.1)
    m = a.gamma >= 0
    assert np.allclose(a.gamma[m] / 3.0, b.gamma[m], rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("perm", list(itertools.permutations(range(3)))[1:])
def test_axis_permutation(pair3, perm):
    p = pair3
    a = oracle.gamma(p.ref, p.eval, p.spacing, 0.02, 2.0, 0.1)
    sp = tuple(p.spacing[i] for i in perm)
    b = oracle.gamma(np.transpose(p.ref, perm), np.transpose(p.eval, perm), sp, 0.02, 2.0, 0.1)
    assert np.allclose(np.transpose(a.gamma, perm), b.gamma, rtol=1e-12, atol=1e-13)


def test_central_inversion(pair3, pair2):
    for p in (pair3, pair2):
        a = oracle.gamma(p.ref, p.eval, p.spacing, 0.02, 2.0, 0.1)
        flip = tuple(slice(None, None, -1) for _ in range(p.ref.ndim))
        b = oracle.gamma(p.ref[flip], p.eval[flip], p.spacing, 0.02, 2.0, 0.1)
        assert np.allclose(a.gamma[flip], b.gamma, rtol=1e-12, atol=1e-13)


def test_extrusion_3d_equals_2d(pair2):
    p = pair2
    a = oracle.gamma(p.ref, p.eval, p.spacing, 0.03, 3.0, 0.1)
    r3 = np.repeat(p.ref[None], 4, axis=0)
    e3 = np.repeat(p.eval[None], 4, axis=0)
    b = oracle.gamma(r3, e3, (2.0,) + p.spacing, 0.03, 3.0, 0.1)
    for z in range(4):
        assert np.allclose(b.gamma[z], a.gamma, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("local", [False, True])
def test_bounds_and_monotonicity(pair3, local):
    p = pair3
    base = oracle.gamma(p.ref, p.eval, p.spacing, 0.02, 2.0, 0.1, local)
    m = base.gamma >= 0
    ref, ev = p.ref.astype(np.float64), p.eval.astype(np.float64)
    dD = 0.02 * (ref if local else ref.max())
    g0 = np.abs(ev - ref) / dD
    assert np.all(base.gamma[m] >= 0)
    assert np.all(base.gamma[m] <= g0[m] + 1e-15)
    more_dd = oracle.gamma(p.ref, p.eval, p.spacing, 0.03, 2.0, 0.1, local)
    more_dta = oracle.gamma(p.ref, p.eval, p.spacing, 0.02, 3.0, 0.1, local)
    assert np.all(more_dd.gamma[m] <= base.gamma[m] + 1e-13)
    assert np.all(more_dta.gamma[m] <= base.gamma[m] + 1e-13)


def _cell_keys(shape, spacing, dta, node):
    """Key of every full grid cell as seen from ``node`` (minimum distance / DTA)."""
    nd = len(shape)
    rng = [np.arange(n - 1) - c for n, c in zip(shape, node)]
    A = np.meshgrid(*rng, indexing="ij")
    s = 0.0
    for i in range(nd):
        g = np.where(A[i] > 0, A[i], np.where(A[i] < -1, -A[i] - 1, 0)).astype(np.float64)
        s = s + (g * spacing[i]) ** 2
    return np.sqrt(s) / dta


def test_work_law(pair3):
    p = pair3
    dta = 2.0
    o = oracle.gamma(p.ref, p.eval, p.spacing, 0.02, dta, 0.1)
    ref, ev = p.ref.astype(np.float64), p.eval.astype(np.float64)
    g0 = np.abs(ev - ref) / (0.02 * ref.max())
    rng = np.random.default_rng(0)
    idx = rng.choice(np.flatnonzero(o.gamma.ravel() >= 0), size=60, replace=False)
    for r in idx:
        node = np.unravel_index(r, p.ref.shape)
        keys = _cell_keys(p.ref.shape, p.spacing, dta, node)
        lo = int(np.sum(keys < o.gamma.ravel()[r]))
        hi = int(np.sum(keys < g0.ravel()[r]))
        assert lo <= o.cells.ravel()[r] <= hi
