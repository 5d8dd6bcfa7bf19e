"""Pin the pruned FP64 oracle to exhaustive search on tiny grids.

The brute force shares no code with the oracle: every face of every simplex of the
whole grid, no table, no early break, Householder QR instead of the normal equations.
Agreement to 1e-10 checks the cell table, its keys, the break rule, the Kuhn
simplices and Ju's recursion at once.
"""
import numpy as np
import pytest

import oracle
from oracle.bruteforce import gamma_bruteforce, kuhn_faces
from dosegen import make_pair_2d, make_pair_3d

TOL = 1e-10


def _rough_pair(seed, shape, amp=0.3):
    """Rough random fields: smooth base + large per-node jumps (many boundary minima)."""
    rng = np.random.default_rng(seed)
    base = rng.uniform(0.2, 1.0, size=shape)
    ref = base + amp * rng.standard_normal(shape)
    ev = ref + amp * rng.standard_normal(shape)
    ref = ref / ref.max()
    return ref.astype(np.float32), ev.astype(np.float32)


def _check(ref, ev, spacing, dd, dta, thr, local):
    o = oracle.gamma(ref, ev, spacing, dd, dta, thr, local)
    b = gamma_bruteforce(ref, ev, spacing, dd, dta, thr, local)
    assert np.array_equal(o.gamma < 0, b < 0), "masks differ"
    m = o.gamma >= 0
    assert m.sum() > 0
    err = np.abs(o.gamma[m] - b[m]).max()
    assert err <= TOL, f"max |oracle - brute| = {err}"
    return o


def test_face_counts_2d_3d():
    # unique faces of the Kuhn lattice: 2D per interior cell 1 vertex, 3 edges, 2 triangles;
    # 3D: 1, 7, 12, 6 (Euler characteristic of the torus is 0).  Full counts on a grid:
    f2 = kuhn_faces((4, 5))
    assert [len(f) for f in f2] == [20, 3 * 12 + 3 + 4, 2 * 12]
    f3 = kuhn_faces((3, 3, 3))
    assert len(f3[0]) == 27 and len(f3[3]) == 6 * 8


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("crit", [(0.03, 3.0, False), (0.01, 1.0, False), (0.02, 2.0, True)])
def test_oracle_vs_bruteforce_2d_smooth(seed, crit):
    p = make_pair_2d(seed, shape=(20, 18), spacing=(1.0, 1.5))
    _check(p.ref, p.eval, p.spacing, crit[0], crit[1], 0.1, crit[2])


@pytest.mark.parametrize("seed", [3, 4])
@pytest.mark.parametrize("spacing", [(1.0, 1.0), (2.0, 0.7)])
@pytest.mark.parametrize("local", [False, True])
def test_oracle_vs_bruteforce_2d_rough(seed, spacing, local):
    ref, ev = _rough_pair(seed, (11, 13))
    _check(ref, ev, spacing, 0.05, 2.0, 0.0, local)


@pytest.mark.parametrize("crit", [(0.03, 3.0, False), (0.01, 1.0, False), (0.02, 2.0, True)])
def test_oracle_vs_bruteforce_3d_smooth(crit):
    p = make_pair_3d(5, shape=(7, 8, 9), spacing=(2.5, 2.0, 2.0))
    _check(p.ref, p.eval, p.spacing, crit[0], crit[1], 0.0, crit[2])


@pytest.mark.parametrize("seed", [6, 7])
@pytest.mark.parametrize("spacing", [(1.0, 1.0, 1.0), (1.5, 0.8, 1.2)])
def test_oracle_vs_bruteforce_3d_rough(seed, spacing):
    ref, ev = _rough_pair(seed, (5, 6, 7))
    _check(ref, ev, spacing, 0.05, 2.0, 0.0, seed == 7)


def test_oracle_subset_matches_full():
    p = make_pair_2d(9, shape=(24, 24))
    full = oracle.gamma(p.ref, p.eval, p.spacing, 0.02, 2.0, 0.1)
    idx = np.array([0, 5, 100, 300, 575, 288, 77])
    sub = oracle.gamma(p.ref, p.eval, p.spacing, 0.02, 2.0, 0.1, subset=idx)
    assert np.array_equal(sub.gamma, full.gamma.ravel()[idx])
    assert np.array_equal(sub.cells, full.cells.ravel()[idx])
