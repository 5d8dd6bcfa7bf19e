"""GPU gamma maps against the FP64 oracle on the same seeded inputs (through the C ABI).

Sizes: the 64x64 2D workload in full; 3D grids from the beam generator small enough for
the oracle to finish in seconds yet spanning many 256-lane tiles with ragged tails; the
full 128x128x96 workload in the benchmark's launch configuration (every node compared);
and a sampled check of the 256x256x192 workload.
"""
import numpy as np
import pytest

import oracle
from dosegen import make_config_pair, make_pair_2d, make_pair_3d
from gpu_util import assert_parity, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gx():
    import paper_1012_1900_amd as g
    return g


@pytest.fixture(scope="module")
def small3d():
    return make_pair_3d(7, shape=(37, 44, 41), spacing=(2.5, 2.5, 2.5))


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_c0_2d(gx, seed):
    p = make_config_pair("c0", seed)
    o = oracle.gamma(p.ref, p.eval, p.spacing, 0.03, 3.0, 0.1)
    g, r = gx.gammax_map(dev(p.ref), dev(p.eval), p.spacing, 0.03, 3.0, 0.1)
    assert_parity(host(g), o.gamma, f"c0 seed {seed}")
    assert r.n_evaluated == o.n_evaluated
    assert abs(int(r.n_pass) - o.n_pass) <= o.n_borderline + r.n_borderline


@pytest.mark.parametrize("crit", [(0.03, 3.0), (0.02, 2.0), (0.01, 1.0)])
@pytest.mark.parametrize("local", [False, True])
def test_small_3d(gx, small3d, crit, local):
    p = small3d
    o = oracle.gamma(p.ref, p.eval, p.spacing, crit[0], crit[1], 0.1, local)
    g, r = gx.gammax_map(dev(p.ref), dev(p.eval), p.spacing, crit[0], crit[1], 0.1, local)
    assert_parity(host(g), o.gamma, f"3d {crit} local={local}")
    assert r.n_evaluated == o.n_evaluated
    assert r.search_radius == pytest.approx(o.radius, rel=1e-6)


def test_anisotropic_3d(gx):
    p = make_pair_3d(8, shape=(23, 31, 29), spacing=(3.0, 2.0, 1.5))
    for crit in [(0.03, 3.0), (0.01, 2.0)]:
        o = oracle.gamma(p.ref, p.eval, p.spacing, crit[0], crit[1], 0.1)
        g, _ = gx.gammax_map(dev(p.ref), dev(p.eval), p.spacing, crit[0], crit[1], 0.1)
        assert_parity(host(g), o.gamma, f"aniso {crit}")


@pytest.mark.parametrize("precision", ["fp32", "guarded", "fp64"])
def test_precision_modes(gx, small3d, precision):
    p = small3d
    o = oracle.gamma(p.ref, p.eval, p.spacing, 0.01, 1.0, 0.1)
    g, r = gx.gammax_map(dev(p.ref), dev(p.eval), p.spacing, 0.01, 1.0, 0.1, precision=precision)
    err = assert_parity(host(g), o.gamma, precision)
    if precision == "fp64":
        # only the final rounding to float32 separates it from the oracle
        m = o.gamma >= 0
        assert np.all(np.abs(host(g)[m] - o.gamma[m]) <= 1e-7 * np.maximum(1.0, o.gamma[m]))
    assert err < 1e-5


def test_guard_forced_everywhere(gx, small3d):
    """cond_threshold = 1 sends every tetrahedron through the FP64 re-projection."""
    p = small3d
    o = oracle.gamma(p.ref, p.eval, p.spacing, 0.02, 2.0, 0.1)
    g, r = gx.gammax_map(dev(p.ref), dev(p.eval), p.spacing, 0.02, 2.0, 0.1, cond_threshold=1.0)
    assert r.n_fp64_tets > 0
    assert_parity(host(g), o.gamma, "forced guard")
    g2, r2 = gx.gammax_map(dev(p.ref), dev(p.eval), p.spacing, 0.02, 2.0, 0.1)
    assert r2.n_fp64_tets == 0
    assert r2.n_cells == r.n_cells


def test_sort_modes_and_determinism(gx, small3d):
    p = small3d
    ref, ev = dev(p.ref), dev(p.eval)
    a, ra = gx.gammax_map(ref, ev, p.spacing, 0.02, 2.0, 0.1, sort="dd")
    b, rb = gx.gammax_map(ref, ev, p.spacing, 0.02, 2.0, 0.1, sort="none")
    c, _ = gx.gammax_map(ref, ev, p.spacing, 0.02, 2.0, 0.1, sort="dd")
    assert np.array_equal(host(a), host(b))
    assert np.array_equal(host(a), host(c))
    assert ra.n_cells == rb.n_cells and ra.n_pass == rb.n_pass


def test_full_c1_bench_configuration(gx):
    """The benchmark workload, every node compared (the oracle takes about a second)."""
    p = make_config_pair("c1", 100)
    o = oracle.gamma(p.ref, p.eval, p.spacing, 0.03, 3.0, 0.1)
    g, r = gx.gammax_map(dev(p.ref), dev(p.eval), p.spacing, 0.03, 3.0, 0.1, timing=True)
    assert_parity(host(g), o.gamma, "c1 3%/3mm")
    assert r.n_evaluated == o.n_evaluated
    assert abs(int(r.n_pass) - o.n_pass) <= o.n_borderline + r.n_borderline
    # visited cells: the same walk up to float rounding at the break
    assert abs(int(r.n_cells) - o.cells_visited) <= 1e-3 * o.cells_visited


def test_c2_sampled(gx):
    """256x256x192 at 1.25 mm: sampled nodes (random plus the largest gamma0) vs the oracle."""
    p = make_config_pair("c2", 200)
    g, r = gx.gammax_map(dev(p.ref), dev(p.eval), p.spacing, 0.02, 2.0, 0.1)
    gh = host(g).ravel()
    rng = np.random.default_rng(5)
    masked = np.flatnonzero(gh >= 0)
    g0 = np.abs(p.eval.ravel()[masked].astype(np.float64) - p.ref.ravel()[masked])
    heavy = masked[np.argsort(g0)[-300:]]
    idx = np.unique(np.concatenate([rng.choice(masked, 3000, replace=False), heavy]))
    o = oracle.gamma(p.ref, p.eval, p.spacing, 0.02, 2.0, 0.1, subset=idx)
    assert_parity(gh[idx], o.gamma, "c2 sampled")
    assert r.n_evaluated == o.n_masked


def test_identical_doses(gx):
    p = make_pair_3d(9, shape=(12, 17, 19), spacing=(2.0, 2.0, 2.0))
    g, r = gx.gammax_map(dev(p.ref), dev(p.ref), p.spacing, 0.03, 3.0, 0.1)
    gh = host(g)
    assert np.all(gh[gh >= 0] == 0.0)
    assert r.n_pass == r.n_evaluated and r.table_len == 0 and r.n_cells == 0


@pytest.mark.parametrize("local", [False, True])
def test_flat_offset_closed_form(gx, local):
    ref = np.full((9, 10, 11), 0.75, dtype=np.float32)
    ev = ref + np.float32(0.0225)
    g, _ = gx.gammax_map(dev(ref), dev(ev), (2.0, 2.0, 2.0), 0.03, 3.0, 0.1, local)
    expect = float(np.float32(0.75) + np.float32(0.0225) - np.float32(0.75)) / (0.03 * 0.75)
    assert np.allclose(host(g), expect, rtol=2e-6, atol=1e-6)


def _rough(seed, shape):
    rng = np.random.default_rng(seed)
    ref = rng.uniform(0.2, 1.0, size=shape) + 0.3 * rng.standard_normal(shape)
    ev = ref + 0.3 * rng.standard_normal(shape)
    return (ref / ref.max()).astype(np.float32), ev.astype(np.float32)


@pytest.mark.parametrize("shape", [(2, 2), (2, 2, 2), (3, 5, 4), (7, 3), (65, 3), (4, 66, 3)])
@pytest.mark.parametrize("local", [False, True])
def test_tiny_and_boundary_heavy(gx, shape, local):
    ref, ev = _rough(len(shape) * 10 + shape[0], shape)
    spacing = tuple(1.0 + 0.5 * i for i in range(len(shape)))
    o = oracle.gamma(ref, ev, spacing, 0.05, 2.0, 0.0, local)
    g, _ = gx.gammax_map(dev(ref), dev(ev), spacing, 0.05, 2.0, 0.0, local)
    assert_parity(host(g), o.gamma, f"rough {shape}")


def test_threshold_edges(gx):
    p = make_pair_2d(21, shape=(50, 70))
    for thr in [0.0, 0.5, 0.99]:
        o = oracle.gamma(p.ref, p.eval, p.spacing, 0.03, 3.0, thr)
        g, r = gx.gammax_map(dev(p.ref), dev(p.eval), p.spacing, 0.03, 3.0, thr)
        assert r.n_evaluated == o.n_evaluated
        assert_parity(host(g), o.gamma, f"thr {thr}")


def test_local_with_no_positive_dose(gx):
    ref = -np.ones((8, 8), dtype=np.float32)
    g, r = gx.gammax_map(dev(ref), dev(ref), (1.0, 1.0), 0.03, 3.0, 0.0, True)
    assert r.n_evaluated == 0 and np.all(host(g) == -1.0)


def test_device_side_errors(gx):
    ref = np.ones((8, 8), dtype=np.float32)
    bad = ref.copy()
    bad[3, 4] = np.nan
    with pytest.raises(gx.GammaxError) as e:
        gx.gammax_map(dev(ref), dev(bad), (1.0, 1.0), 0.03, 3.0, 0.1)
    assert e.value.status == -4
    with pytest.raises(gx.GammaxError) as e:
        gx.gammax_map(dev(-ref), dev(ref), (1.0, 1.0), 0.03, 3.0, 0.1)
    assert e.value.status == -8
    # the context stays usable after an error
    g, r = gx.gammax_map(dev(ref), dev(ref), (1.0, 1.0), 0.03, 3.0, 0.1)
    assert r.n_evaluated == 64


def test_flat_entry_point(gx):
    p = make_config_pair("c0", 4)
    a, pr = gx.gamma_map(dev(p.ref), dev(p.eval), p.spacing, 0.03, 3.0, 0.1)
    b, r = gx.gammax_map(dev(p.ref), dev(p.eval), p.spacing, 0.03, 3.0, 0.1)
    assert np.array_equal(host(a), host(b))
    assert pr == pytest.approx(r.pass_rate)
