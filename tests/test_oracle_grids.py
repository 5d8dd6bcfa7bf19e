"""Pins of the two-grid oracle (the evaluation dose on a grid of its own): the one-grid
oracle at zero offset and equal spacing, closed forms on shifted and refined grids (an
exactly represented linear dose, a flat offset, a shifted ramp's point-to-plane distance),
and nodes outside the evaluation grid's box."""
import numpy as np
import pytest

import oracle
from dosegen import make_pair_3d


def test_same_grid_matches_one_grid_oracle():
    p = make_pair_3d(3, shape=(17, 19, 21), spacing=(2.5, 2.0, 3.0))
    for crit, local in (((0.03, 3.0), False), ((0.02, 2.0), True)):
        a = oracle.gamma(p.ref, p.eval, p.spacing, crit[0], crit[1], 0.1, local)
        b = oracle.gamma_grids(p.ref, p.eval, p.spacing, p.spacing, (0.0, 0.0, 0.0), crit[0], crit[1], 0.1, local)
        assert a.n_evaluated == b.n_evaluated
        m = a.gamma >= 0
        assert np.array_equal(m, b.gamma >= 0)
        assert np.allclose(b.gamma[m], a.gamma[m], rtol=1e-12, atol=1e-12)


def _grid(shape, spacing, origin=(0.0, 0.0, 0.0)):
    return np.meshgrid(*[o + h * np.arange(n) for n, h, o in zip(shape, spacing, origin)], indexing="ij")


@pytest.mark.parametrize("ev_spacing,ev_origin", [((2.0, 2.0, 2.0), (0.7, -1.3, 0.4)),
                                                   ((1.0, 1.5, 0.8), (-2.0, -2.0, -2.0)),
                                                   ((4.0, 3.0, 5.0), (-5.0, -3.0, -5.0))])
def test_linear_dose_is_represented_exactly(ev_spacing, ev_origin):
    """A linear dose sampled on any grid is its own PL interpolant: gamma = 0 inside."""
    ref_sp = (2.0, 2.0, 2.0)
    lin = lambda z, y, x: 1.0 + 0.02 * z - 0.015 * y + 0.01 * x  # noqa: E731
    ref = lin(*_grid((12, 13, 14), ref_sp))
    ev_shape = tuple(int(np.ceil((n * 2.0 + 6.0) / h)) for n, h in zip((12, 13, 14), ev_spacing))
    ev = lin(*_grid(ev_shape, ev_spacing, ev_origin))
    o = oracle.gamma_grids(ref, ev, ref_sp, ev_spacing, ev_origin, 0.03, 3.0, 0.0)
    m = o.gamma >= 0
    assert m.sum() > 0.5 * m.size
    assert np.all(o.gamma[m] <= 1e-9)


def test_flat_offset_on_a_shifted_grid():
    ref = np.full((9, 10, 11), 2.0)
    ev = np.full((12, 12, 12), 2.0 + 0.05)
    o = oracle.gamma_grids(ref, ev, (1.0, 1.0, 1.0), (0.9, 0.9, 0.9), (-0.35, -0.2, -0.6), 0.03, 3.0, 0.1)
    m = o.gamma >= 0
    assert m.sum() > 0
    assert np.allclose(o.gamma[m], 0.05 / (0.03 * 2.0), rtol=1e-12)


def test_shifted_ramp_point_to_plane():
    """Reference ramp a + b x on one grid, the same ramp shifted by s on a finer, offset
    grid: gamma = |b s| / dD / sqrt(1 + (b DTA / dD)^2) wherever the foot of the
    perpendicular lies inside the evaluation grid."""
    a, b, s = 1.0, 0.01, 1.7   # dose per mm, shift in mm
    ref_sp, ev_sp, ev_o = (2.0, 2.0, 2.0), (1.25, 1.25, 1.25), (-10.0, -10.0, -10.0)
    z, y, x = _grid((8, 9, 30), ref_sp)
    ref = a + b * x
    ez, ey, ex = _grid((30, 30, 70), ev_sp, ev_o)
    ev = a + b * (ex - s)
    dd, dta = 0.03, 3.0
    o = oracle.gamma_grids(ref, ev, ref_sp, ev_sp, ev_o, dd, dta, 0.0)
    dD = dd * ref.max()
    want = abs(b * s) / dD / np.sqrt(1.0 + (b * dta / dD) ** 2)
    inner = (o.gamma >= 0) & (x > 10.0) & (x < 50.0)
    assert inner.sum() > 100
    assert np.allclose(o.gamma[inner], want, rtol=1e-10)


def test_nodes_outside_the_evaluation_box():
    ref = np.full((6, 6, 6), 1.0)
    ev = np.full((4, 4, 4), 1.0)
    o = oracle.gamma_grids(ref, ev, (1.0, 1.0, 1.0), (1.0, 1.0, 1.0), (1.0, 1.0, 1.0), 0.03, 3.0, 0.1)
    inside = np.zeros((6, 6, 6), dtype=bool)
    inside[1:5, 1:5, 1:5] = True
    assert np.array_equal(o.gamma >= 0, inside)
    assert np.all(o.gamma[inside] == 0.0)
    assert o.n_evaluated == inside.sum() and o.n_masked == 216


# ---- 2D --------------------------------------------------------------------------------

def test_2d_same_grid_matches_one_grid_oracle():
    from dosegen import make_pair_2d
    p = make_pair_2d(4, shape=(40, 44), spacing=(1.0, 1.5))
    for crit, local in (((0.03, 3.0), False), ((0.02, 2.0), True)):
        a = oracle.gamma(p.ref, p.eval, p.spacing, crit[0], crit[1], 0.1, local)
        b = oracle.gamma_grids(p.ref, p.eval, p.spacing, p.spacing, (0.0, 0.0), crit[0], crit[1], 0.1, local)
        assert a.n_evaluated == b.n_evaluated
        m = a.gamma >= 0
        assert np.array_equal(m, b.gamma >= 0)
        assert np.allclose(b.gamma[m], a.gamma[m], rtol=1e-12, atol=1e-12)


def test_2d_linear_dose_and_shifted_ramp():
    """A linear dose on any 2D grid is its own interpolant (gamma = 0 inside), and a ramp
    shifted by s on a finer offset grid gives the point-to-line distance."""
    lin = lambda y, x: 1.0 - 0.015 * y + 0.01 * x  # noqa: E731
    ref_sp, ev_sp, ev_o = (2.0, 2.0), (1.3, 0.7), (-1.1, 0.45)
    ref = lin(*_grid((13, 14), ref_sp, (0.0, 0.0)))
    ev = lin(*_grid((24, 44), ev_sp, ev_o))
    o = oracle.gamma_grids(ref, ev, ref_sp, ev_sp, ev_o, 0.03, 3.0, 0.0)
    m = o.gamma >= 0
    assert m.sum() > 0.5 * m.size and np.all(o.gamma[m] <= 1e-9)
    a, b, s, dd, dta = 1.0, 0.01, 1.7, 0.03, 3.0
    y, x = _grid((9, 30), (2.0, 2.0), (0.0, 0.0))
    ey, ex = _grid((30, 70), (1.25, 1.25), (-10.0, -10.0))
    o = oracle.gamma_grids(a + b * x, a + b * (ex - s), (2.0, 2.0), (1.25, 1.25), (-10.0, -10.0), dd, dta, 0.0)
    dD = dd * (a + b * x).max()
    want = abs(b * s) / dD / np.sqrt(1.0 + (b * dta / dD) ** 2)
    inner = (o.gamma >= 0) & (x > 10.0) & (x < 50.0)
    assert inner.sum() > 50
    assert np.allclose(o.gamma[inner], want, rtol=1e-10)


def test_2d_equals_its_3d_extrusion():
    """A pair constant along an added slowest axis gives the 2D gamma in every layer: the
    3D Kuhn interpolant of such a dose is the 2D interpolant at every height."""
    from dosegen import make_pair_2d
    p = make_pair_2d(5, shape=(30, 33), spacing=(1.0, 1.0))
    ev_sp, ev_o = (0.8, 1.3), (0.25, -0.4)
    shape = tuple(int(round(n * h / e)) for n, h, e in zip(p.ref.shape, p.spacing, ev_sp))
    ev = make_pair_2d(5, shape=shape, spacing=ev_sp).eval
    o2 = oracle.gamma_grids(p.ref, ev, p.spacing, ev_sp, ev_o, 0.03, 3.0, 0.1)
    ref3 = np.stack([p.ref, p.ref])
    ev3 = np.stack([ev, ev, ev])
    o3 = oracle.gamma_grids(ref3, ev3, (1.7,) + p.spacing, (0.85,) + ev_sp, (0.0,) + ev_o, 0.03, 3.0, 0.1)
    for layer in range(2):
        m = o2.gamma >= 0
        assert np.array_equal(m, o3.gamma[layer] >= 0)
        assert np.allclose(o3.gamma[layer][m], o2.gamma[m], rtol=1e-10, atol=1e-12)
