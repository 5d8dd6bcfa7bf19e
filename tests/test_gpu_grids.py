"""GPU tests of gammax_map_grids (the evaluation dose on a grid of its own): the two-grid
FP64 oracle within the bar for offset, finer, coarser and anisotropic evaluation grids,
global and local, in every precision; the one-grid map at zero offset and equal spacing;
closed forms (an exactly represented linear dose, a flat offset); nodes outside the
evaluation box; refused options."""
import numpy as np
import pytest

import oracle
from dosegen import make_pair_3d
from gpu_util import assert_parity, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gx():
    import paper_1012_1900_amd as g
    return g


def _eval_on(seed, ref_shape, ref_sp, ev_sp, shift):
    """The generator's evaluation dose on another grid over the same box (the generator
    centres its axes), the sampling positions moved by `shift` mm; returns it with the
    evaluation grid's origin in the reference frame."""
    shape = tuple(max(2, int(round(n * h / e))) for n, h, e in zip(ref_shape, ref_sp, ev_sp))
    p = make_pair_3d(seed, shape=shape, spacing=ev_sp)
    origin = tuple((n - 1) / 2 * h - (m - 1) / 2 * e + d
                   for n, h, m, e, d in zip(ref_shape, ref_sp, shape, ev_sp, shift))
    return p.eval.astype(np.float32), origin


CASES = [
    ((2.5, 2.5, 2.5), (0.9, -1.1, 0.6)),      # same spacing, offset
    ((1.25, 1.25, 1.25), (0.0, 0.0, 0.0)),    # twice as fine
    ((5.0, 5.0, 5.0), (-2.0, 1.0, -3.0)),     # twice as coarse, offset
    ((2.0, 3.0, 1.5), (-1.0, -0.5, 0.25)),    # anisotropic
]


@pytest.mark.parametrize("ev_sp,ev_o", CASES)
@pytest.mark.parametrize("local", [False, True])
def test_grids_match_the_oracle(gx, ev_sp, ev_o, local):
    ref_sp = (2.5, 2.5, 2.5)
    p = make_pair_3d(51, shape=(18, 21, 20), spacing=ref_sp)
    ev, ev_o = _eval_on(51, p.ref.shape, ref_sp, ev_sp, ev_o)
    o = oracle.gamma_grids(p.ref, ev, ref_sp, ev_sp, ev_o, 0.03, 3.0, 0.1, local)
    g, r = gx.gammax_map_grids(dev(p.ref), dev(ev), ref_sp, ev_sp, ev_o, 0.03, 3.0, 0.1, local)
    assert_parity(host(g), o.gamma, f"grids {ev_sp} {ev_o} local={local}")
    assert r.n_evaluated == o.n_evaluated > 0
    assert abs(int(r.n_pass) - o.n_pass) <= o.n_borderline + r.n_borderline


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_grids_precisions(gx, precision):
    ref_sp, ev_sp, ev_o = (2.5, 2.5, 2.5), (2.0, 2.0, 2.0), (0.3, 0.7, -0.4)
    p = make_pair_3d(52, shape=(16, 17, 18), spacing=ref_sp)
    ev, ev_o = _eval_on(52, p.ref.shape, ref_sp, ev_sp, ev_o)
    o = oracle.gamma_grids(p.ref, ev, ref_sp, ev_sp, ev_o, 0.02, 2.0, 0.1)
    g, r = gx.gammax_map_grids(dev(p.ref), dev(ev), ref_sp, ev_sp, ev_o, 0.02, 2.0, 0.1, precision=precision)
    assert_parity(host(g), o.gamma, f"grids {precision}")


def test_same_grid_equals_gammax_map(gx):
    p = make_pair_3d(53, shape=(20, 22, 19), spacing=(2.5, 2.0, 3.0))
    g1, r1 = gx.gammax_map(dev(p.ref), dev(p.eval), p.spacing, 0.03, 3.0, 0.1)
    g2, r2 = gx.gammax_map_grids(dev(p.ref), dev(p.eval), p.spacing, p.spacing, (0.0, 0.0, 0.0), 0.03, 3.0, 0.1)
    a, b = host(g1), host(g2)
    assert np.array_equal(a >= 0, b >= 0)
    m = a >= 0
    assert np.all(np.abs(a[m] - b[m]) <= 1e-5 + 1e-5 * a[m])
    assert r1.n_evaluated == r2.n_evaluated


def test_closed_forms_and_outside_nodes(gx):
    ref_sp, ev_sp, ev_o = (2.0, 2.0, 2.0), (1.5, 1.25, 1.75), (-0.8, 0.3, -1.1)
    z, y, x = np.meshgrid(*[np.arange(n) * h for n, h in zip((10, 11, 12), ref_sp)], indexing="ij")
    lin = lambda z, y, x: 1.0 + 0.02 * z - 0.015 * y + 0.01 * x  # noqa: E731
    ref = lin(z, y, x).astype(np.float32)
    es = (14, 17, 14)
    ez, ey, ex = np.meshgrid(*[o + np.arange(n) * h for n, h, o in zip(es, ev_sp, ev_o)], indexing="ij")
    ev = lin(ez, ey, ex).astype(np.float32)
    g, r = gx.gammax_map_grids(dev(ref), dev(ev), ref_sp, ev_sp, ev_o, 0.03, 3.0, 0.0)
    gh = host(g)
    u = [(c - o) / h for c, o, h in zip((z, y, x), ev_o, ev_sp)]
    inside = np.all([(ui >= 0) & (ui <= n - 1) for ui, n in zip(u, es)], axis=0)
    assert np.array_equal(gh >= 0, inside) and inside.sum() > 100
    assert np.all(gh[inside] <= 1e-3)   # float32 doses of a linear field: gamma ~ 0
    # flat offset: gamma = delta / dD everywhere inside
    ref2 = np.full((10, 11, 12), 2.0, np.float32)
    ev2 = np.full(es, 2.05, np.float32)
    g2, _ = gx.gammax_map_grids(dev(ref2), dev(ev2), ref_sp, ev_sp, ev_o, 0.03, 3.0, 0.1)
    g2h = host(g2)
    assert np.allclose(g2h[inside], 0.05 / (0.03 * 2.0), rtol=2e-5)


@pytest.mark.parametrize("precision", ["guarded", "fp32", "fp64"])
def test_identical_doses_on_the_same_grid(gx, precision):
    """Every first bound is 0 (the evaluation dose equals the reference at every node, on the
    same grid): no table is needed, and every evaluated node has gamma 0 and passes."""
    p = make_pair_3d(57, shape=(12, 14, 13), spacing=(2.5, 2.5, 2.5))
    g, r = gx.gammax_map_grids(dev(p.ref), dev(p.ref), p.spacing, p.spacing, (0.0, 0.0, 0.0), 0.03, 3.0, 0.1,
                               precision=precision)
    o = oracle.gamma(p.ref, p.ref, p.spacing, 0.03, 3.0, 0.1)
    gh = host(g)
    assert np.array_equal(gh >= 0, o.gamma >= 0) and r.n_evaluated > 0
    assert np.all(gh[gh >= 0] == 0.0)
    assert r.n_pass == r.n_evaluated


def test_cached_table_and_a_radius_that_outgrows_it(gx):
    """On one context the table built for the first map serves the next ones of the same
    geometry (one read-back per map); a map whose radius outgrows it runs again on a larger
    one.  Every map equals the same map on a fresh context bit for bit."""
    ref_sp, ev_sp, ev_o = (2.5, 2.5, 2.5), (2.5, 2.5, 2.5), (1.25, -0.5, 0.75)
    p = make_pair_3d(58, shape=(16, 18, 17), spacing=ref_sp)
    ev_small = p.ref + np.float32(0.3) * (p.eval - p.ref)
    ev_large = p.ref + np.float32(3.0) * (p.eval - p.ref)
    ctx = gx.Context(0)
    for ev in (ev_small, ev_large, ev_small, ev_large):
        g, r = gx.gammax_map_grids(dev(p.ref), dev(ev), ref_sp, ev_sp, ev_o, 0.03, 3.0, 0.1, ctx=ctx)
        g0, r0 = gx.gammax_map_grids(dev(p.ref), dev(ev), ref_sp, ev_sp, ev_o, 0.03, 3.0, 0.1, ctx=gx.Context(0))
        assert np.array_equal(host(g), host(g0))
        assert (r.n_evaluated, r.n_pass) == (r0.n_evaluated, r0.n_pass)
    o = oracle.gamma_grids(p.ref, ev_large, ref_sp, ev_sp, ev_o, 0.03, 3.0, 0.1)
    assert_parity(host(g), o.gamma, "cached table, large radius")


def test_refused_options(gx):
    p = make_pair_3d(54, shape=(8, 9, 10), spacing=(2.5, 2.5, 2.5))
    with pytest.raises(gx.GammaxError) as e:
        gx.gammax_map_grids(dev(p.ref), dev(p.eval), p.spacing, p.spacing, (0, 0, 0), 0.03, 3.0, tail_lanes=1)
    assert e.value.status == -3


def _eval_on_2d(seed, ref_shape, ref_sp, ev_sp, shift):
    """The 2D generator's evaluation dose on another grid over the same field (centred axes),
    the sampling positions moved by `shift` mm; with the evaluation grid's origin."""
    from dosegen import make_pair_2d
    shape = tuple(max(2, int(round(n * h / e))) for n, h, e in zip(ref_shape, ref_sp, ev_sp))
    p = make_pair_2d(seed, shape=shape, spacing=ev_sp)
    origin = tuple((n - 1) / 2 * h - (m - 1) / 2 * e + d
                   for n, h, m, e, d in zip(ref_shape, ref_sp, shape, ev_sp, shift))
    return p.eval.astype(np.float32), origin


CASES_2D = [
    ((1.0, 1.0), (0.35, -0.45)),     # same spacing, offset
    ((0.5, 0.5), (0.0, 0.0)),        # twice as fine
    ((2.0, 2.0), (-0.7, 0.9)),       # twice as coarse, offset
    ((0.8, 1.3), (0.2, -0.6)),       # anisotropic
]


@pytest.mark.parametrize("ev_sp,ev_o", CASES_2D)
@pytest.mark.parametrize("local", [False, True])
def test_grids_2d_match_the_oracle(gx, ev_sp, ev_o, local):
    from dosegen import make_pair_2d
    ref_sp = (1.0, 1.0)
    p = make_pair_2d(61, shape=(48, 52), spacing=ref_sp)
    ev, ev_o = _eval_on_2d(61, p.ref.shape, ref_sp, ev_sp, ev_o)
    o = oracle.gamma_grids(p.ref, ev, ref_sp, ev_sp, ev_o, 0.03, 3.0, 0.1, local)
    g, r = gx.gammax_map_grids(dev(p.ref), dev(ev), ref_sp, ev_sp, ev_o, 0.03, 3.0, 0.1, local)
    assert g.shape == p.ref.shape
    assert_parity(host(g), o.gamma, f"2D grids {ev_sp} {ev_o} local={local}")
    assert r.n_evaluated == o.n_evaluated > 0
    assert abs(int(r.n_pass) - o.n_pass) <= o.n_borderline + r.n_borderline


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_grids_2d_same_grid_equals_gammax_map(gx, precision):
    from dosegen import make_pair_2d
    p = make_pair_2d(62, shape=(40, 45), spacing=(1.0, 1.5))
    g1, r1 = gx.gammax_map(dev(p.ref), dev(p.eval), p.spacing, 0.02, 2.0, 0.1, precision=precision)
    g2, r2 = gx.gammax_map_grids(dev(p.ref), dev(p.eval), p.spacing, p.spacing, (0.0, 0.0), 0.02, 2.0, 0.1,
                                 precision=precision)
    a, b = host(g1), host(g2)
    assert np.array_equal(a >= 0, b >= 0)
    m = a >= 0
    assert np.all(np.abs(a[m] - b[m]) <= 1e-5 + 1e-5 * a[m])
    assert (r1.n_evaluated, r1.n_pass) == (r2.n_evaluated, r2.n_pass)
