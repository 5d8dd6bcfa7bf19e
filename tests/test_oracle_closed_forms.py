"""Closed forms that pin the oracle (Eq. (1) with the geometric method of Sec. 2.1).

* identical doses: gamma = 0;
* flat field c, evaluation c + delta: the surface is the plane D = c + delta, so
  gamma = |delta| / dD, with dD = DD * c under both global and local normalisation;
* linear ramp D_r = a.x + b, D_e(x) = D_r(x - s): Kuhn interpolation reproduces linear
  functions, the surface is a hyperplane, and gamma = |a.s| / sqrt(dD^2 + DTA^2 |a|^2)
  wherever the foot point stays over the grid box;
* point-to-simplex distances with known answers (the projection formula of Sec. 2.1).
"""
import math

import numpy as np
import pytest

import oracle


def test_identical_doses_give_zero():
    rng = np.random.default_rng(1)
    ref = rng.uniform(0, 1, size=(6, 7, 8)).astype(np.float32)
    o = oracle.gamma(ref, ref, (1.0, 2.0, 3.0), 0.03, 3.0, 0.1)
    m = o.gamma >= 0
    assert m.sum() == o.n_evaluated > 0
    assert np.all(o.gamma[m] == 0.0)
    assert o.cells_visited == 0          # radius 0: nothing to walk
    assert o.n_pass == o.n_evaluated


@pytest.mark.parametrize("local", [False, True])
@pytest.mark.parametrize("shape,spacing", [((9, 11), (1.0, 1.5)), ((5, 6, 7), (2.5, 1.0, 2.0))])
@pytest.mark.parametrize("delta", [0.004, -0.025, 0.11])
def test_flat_offset(local, shape, spacing, delta):
    c = 0.75
    ref = np.full(shape, c)
    ev = ref + delta
    dd = 0.03
    o = oracle.gamma(ref, ev, spacing, dd, 3.0, 0.1, local)
    expect = abs(delta) / (dd * c)
    assert np.allclose(o.gamma, expect, rtol=1e-13, atol=1e-13)


def _ramp_case(shape, spacing, a, s, dd, dta, margin_mm):
    nd = len(shape)
    axes = [np.arange(n, dtype=np.float64) * h for n, h in zip(shape, spacing)]
    X = np.meshgrid(*axes, indexing="ij")
    lin = sum(ai * Xi for ai, Xi in zip(a, X))
    ref = 0.5 + lin
    ev = 0.5 + lin - float(np.dot(a, s))
    dD = dd * ref.max()
    expect = abs(float(np.dot(a, s))) / math.sqrt(dD ** 2 + dta ** 2 * float(np.dot(a, a)))
    o = oracle.gamma(ref, ev, spacing, dd, dta, 0.0, False)
    # interior nodes: foot point (within expect*dta of the node) stays over the grid box
    inner = np.ones(shape, dtype=bool)
    for i in range(nd):
        k = int(math.ceil(margin_mm / spacing[i]))
        lo = [slice(None)] * nd
        lo[i] = slice(0, k)
        hi = [slice(None)] * nd
        hi[i] = slice(shape[i] - k, None)
        inner[tuple(lo)] = False
        inner[tuple(hi)] = False
    assert inner.sum() > 0
    return o, expect, inner


@pytest.mark.parametrize("a,s", [((0.02, 0.0), (1.0, 0.0)), ((0.01, -0.015), (0.7, 1.3)),
                                 ((-0.03, 0.004), (-2.0, 0.5))])
def test_ramp_shift_2d(a, s):
    shape, spacing = (21, 23), (1.0, 1.25)
    o, expect, inner = _ramp_case(shape, spacing, np.array(a), np.array(s), 0.03, 3.0, 6.0)
    assert np.allclose(o.gamma[inner], expect, rtol=1e-12, atol=1e-12)
    edge = (~inner) & (o.gamma >= 0)
    assert np.all(o.gamma[edge] >= expect - 1e-12)   # the box edge can only cut the surface


@pytest.mark.parametrize("a,s", [((0.01, 0.02, -0.005), (0.5, -1.0, 1.5)),
                                 ((0.0, 0.0, 0.04), (0.0, 0.0, 2.2)),
                                 ((-0.015, 0.01, 0.01), (1.2, 1.2, -0.4))])
def test_ramp_shift_3d(a, s):
    shape, spacing = (11, 12, 13), (2.0, 1.5, 1.0)
    o, expect, inner = _ramp_case(shape, spacing, np.array(a), np.array(s), 0.02, 2.5, 6.0)
    assert np.allclose(o.gamma[inner], expect, rtol=1e-12, atol=1e-12)


def test_simplex_distances_known():
    sd = oracle.simplex_dist
    # vertex
    assert sd(np.array([[3.0, 4.0]])) == pytest.approx(5.0)
    # segment, projection inside / beyond an end
    assert sd(np.array([[1.0, -1.0], [1.0, 1.0]])) == pytest.approx(1.0)
    assert sd(np.array([[1.0, 1.0], [2.0, 3.0]])) == pytest.approx(math.sqrt(2.0))
    # triangle: projection at the centroid
    assert sd(np.eye(3)) == pytest.approx(1.0 / math.sqrt(3.0))
    # triangle whose closest point is a vertex
    assert sd(np.array([[1.0, 1.0, 0.0], [2.0, 1.0, 0.0], [1.0, 2.0, 0.0]])) == pytest.approx(math.sqrt(2.0))
    # triangle whose closest point is inside an edge
    assert sd(np.array([[1.0, -1.0, 0.0], [1.0, 1.0, 0.0], [3.0, 0.0, 0.0]])) == pytest.approx(1.0)
    # tetrahedron in 4D: the standard simplex, projection at the centroid
    assert sd(np.eye(4)) == pytest.approx(0.5)
    # lifted tetrahedron at dose height 5 whose spatial closest point lies on a facet
    v = np.array([[1, 0, 0, 5], [0, 1, 0, 5], [0, 0, 1, 5], [1, 1, 1, 5]], dtype=float)
    assert sd(v) == pytest.approx(math.sqrt(25.0 + 1.0 / 3.0))
