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
    p = make_config_pair("2d_64x64_1mm", seed)
    o = oracle.gamma(p.ref, p.eval, p.spacing, 0.03, 3.0, 0.1)
    g, r = gx.gammax_map(dev(p.ref), dev(p.eval), p.spacing, 0.03, 3.0, 0.1)
    assert_parity(host(g), o.gamma, f"2D 64x64 seed {seed}")
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


@pytest.mark.parametrize("precision", ["fp32", "guarded"])
@pytest.mark.parametrize("local", [False, True])
def test_ju_recursion_projection(gx, small3d, precision, local):
    """Ju et al.'s recursion in the key-0 pass (projection="ju"): the oracle's gamma within
    the bar, on isotropic and anisotropic grids, with the pass decisions of the default."""
    for p, crit in ((small3d, (0.02, 2.0)), (make_pair_3d(8, shape=(23, 31, 29), spacing=(3.0, 2.0, 1.5)), (0.03, 3.0))):
        o = oracle.gamma(p.ref, p.eval, p.spacing, crit[0], crit[1], 0.1, local)
        g, r = gx.gammax_map(dev(p.ref), dev(p.eval), p.spacing, crit[0], crit[1], 0.1, local, precision=precision,
                             projection="ju")
        assert_parity(host(g), o.gamma, f"ju {crit} local={local} {precision}")
        g0, r0 = gx.gammax_map(dev(p.ref), dev(p.eval), p.spacing, crit[0], crit[1], 0.1, local, precision=precision)
        assert r.n_evaluated == r0.n_evaluated
        assert abs(int(r.n_pass) - int(r0.n_pass)) <= r.n_borderline + r0.n_borderline


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
    g2, r2 = gx.gammax_map(dev(p.ref), dev(p.eval), p.spacing, 0.02, 2.0, 0.1, tail_lanes=1)
    assert r2.n_fp64_tets == 0 and r2.n_guarded == 0
    assert r.n_guarded == r.n_evaluated
    assert r2.n_cells == r.n_cells   # the same sequential walk, FP64 or not


def test_sort_modes_and_determinism(gx, small3d):
    p = small3d
    ref, ev = dev(p.ref), dev(p.eval)
    a, ra = gx.gammax_map(ref, ev, p.spacing, 0.02, 2.0, 0.1, sort="dd")
    b, rb = gx.gammax_map(ref, ev, p.spacing, 0.02, 2.0, 0.1, sort="none")
    c, _ = gx.gammax_map(ref, ev, p.spacing, 0.02, 2.0, 0.1, sort="dd")
    d, rd = gx.gammax_map(ref, ev, p.spacing, 0.02, 2.0, 0.1, sort="bound")
    assert np.array_equal(host(a), host(b))
    assert np.array_equal(host(a), host(c))
    assert np.array_equal(host(a), host(d))
    assert ra.n_cells == rb.n_cells == rd.n_cells and ra.n_pass == rb.n_pass == rd.n_pass
    assert ra.n_tail > 0 and ra.n_tail == rb.n_tail


@pytest.mark.parametrize("kind", ["3d", "2d"])
def test_given_order(gx, small3d, kind):
    """A caller's key orders the walk past the key-0 cells; gamma, counts and the tail are
    those of the unsorted walk whatever the key: the true gamma, noise, or negative and NaN
    keys (which count as 0)."""
    import torch
    p = small3d if kind == "3d" else make_config_pair("2d_64x64_1mm", 5)
    ref, ev = dev(p.ref), dev(p.eval)
    crit = (0.02, 2.0) if kind == "3d" else (0.01, 1.0)
    base, rb = gx.gammax_map(ref, ev, p.spacing, *crit, 0.1, sort="none")
    assert rb.n_tail > 0
    gen = torch.Generator(device=ref.device).manual_seed(3)
    noise = torch.rand(ref.shape, generator=gen, device=ref.device)
    odd = noise - 0.5
    odd.view(-1)[::7] = float("nan")
    for key in (base.clone(), noise, odd):
        g, r = gx.gammax_map(ref, ev, p.spacing, *crit, 0.1, sort="given", order_key=key)
        assert np.array_equal(host(g), host(base))
        assert (r.n_cells, r.n_pass, r.n_tail, r.n_guarded) == (rb.n_cells, rb.n_pass, rb.n_tail, rb.n_guarded)
    # queued, twice with the same key (both on the cached table)
    for _ in range(2):
        t = gx.gammax_map_async(ref, ev, p.spacing, *crit, 0.1, sort="given", order_key=noise)
        r = t.wait()
        assert np.array_equal(host(t.gamma), host(base)) and r.n_cells == rb.n_cells


def test_given_order_refusals(gx, small3d):
    p = small3d
    ref, ev = dev(p.ref), dev(p.eval)
    with pytest.raises(gx.GammaxError):
        gx.gammax_map(ref, ev, p.spacing, 0.03, 3.0, 0.1, sort="given")
    with pytest.raises(ValueError):
        gx.gammax_map(ref, ev, p.spacing, 0.03, 3.0, 0.1, sort="given", order_key=ref[:1].contiguous())
    with pytest.raises(gx.GammaxError):
        gx.gammax_map(ref, ev, p.spacing, 0.03, 3.0, 0.1, sort="given", order_key=ref, radius="learned")
    with pytest.raises(gx.GammaxError):
        gx.gammax_map_many([dict(ref=ref, ev=ev, spacing=p.spacing, dd=0.03, dta=3.0)], sort="given")


def test_full_c1_bench_configuration(gx):
    """The benchmark workload, every node compared (the oracle takes about a second)."""
    p = make_config_pair("3d_128x128x96_2.5mm", 100)
    o = oracle.gamma(p.ref, p.eval, p.spacing, 0.03, 3.0, 0.1)
    g, r = gx.gammax_map(dev(p.ref), dev(p.eval), p.spacing, 0.03, 3.0, 0.1, timing=True)
    assert_parity(host(g), o.gamma, "128x128x96 3%/3mm")
    assert r.n_evaluated == o.n_evaluated
    assert abs(int(r.n_pass) - o.n_pass) <= o.n_borderline + r.n_borderline
    # visited cells: every cell of the exact walk (up to float rounding at the break); the
    # cooperative tail walk may evaluate up to lanes-1 more per tail node
    assert o.cells_visited * (1 - 1e-4) <= r.n_cells <= o.cells_visited + 63 * r.n_tail
    for lanes in (1, 8, 64):
        g2, r2 = gx.gammax_map(dev(p.ref), dev(p.eval), p.spacing, 0.03, 3.0, 0.1, tail_lanes=lanes)
        assert np.array_equal(host(g2), host(g))
        if lanes == 1:
            assert abs(int(r2.n_cells) - o.cells_visited) <= 1e-4 * o.cells_visited


def test_c2_sampled(gx):
    """256x256x192 at 1.25 mm: sampled nodes (random plus the largest gamma0) vs the oracle."""
    p = make_config_pair("3d_256x256x192_1.25mm", 200)
    g, r = gx.gammax_map(dev(p.ref), dev(p.eval), p.spacing, 0.02, 2.0, 0.1)
    gh = host(g).ravel()
    rng = np.random.default_rng(5)
    masked = np.flatnonzero(gh >= 0)
    g0 = np.abs(p.eval.ravel()[masked].astype(np.float64) - p.ref.ravel()[masked])
    heavy = masked[np.argsort(g0)[-300:]]
    idx = np.unique(np.concatenate([rng.choice(masked, 3000, replace=False), heavy]))
    o = oracle.gamma(p.ref, p.eval, p.spacing, 0.02, 2.0, 0.1, subset=idx)
    assert_parity(gh[idx], o.gamma, "256x256x192 sampled")
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


@pytest.mark.parametrize("shape", [(13, 64, 80), (33, 96, 100)])
def test_prep_partial_tile_group(gx, shape):
    """Grids whose prep tiles (1024 nodes) do not fill the last tile group: 65 tiles in
    groups of 2, 310 tiles in groups of 4.  The compaction's order and count, R and every
    gamma must still match the oracle."""
    p = make_pair_3d(31, shape=shape, spacing=(2.5, 2.5, 2.5))
    o = oracle.gamma(p.ref, p.eval, p.spacing, 0.03, 3.0, 0.1)
    g, r = gx.gammax_map(dev(p.ref), dev(p.eval), p.spacing, 0.03, 3.0, 0.1)
    assert_parity(host(g), o.gamma, f"partial tile group {shape}")
    assert r.n_evaluated == o.n_evaluated
    assert r.search_radius == pytest.approx(o.radius, rel=1e-6)


def test_long_walks_widen_the_tail(gx):
    """A local-normalised pair whose longest tail walks run to thousands of table rows: the
    first map records the longest walk, the next map of the context walks its tail in
    wider lane groups.  Both match the oracle."""
    p = make_pair_3d(40064, shape=(32, 48, 48), spacing=(1.0, 1.0, 1.0))
    o = oracle.gamma(p.ref, p.eval, p.spacing, 0.03, 3.0, 0.1, True)
    ctx = gx.Context(0)
    ref, ev = dev(p.ref), dev(p.eval)
    g1, r1 = gx.gammax_map(ref, ev, p.spacing, 0.03, 3.0, 0.1, True, ctx=ctx)
    g1 = host(g1)
    g2, r2 = gx.gammax_map(ref, ev, p.spacing, 0.03, 3.0, 0.1, True, ctx=ctx)
    assert r1.long_walk_rows > 256 and r2.long_walk_rows > 256
    for g, lab in ((g1, "first map"), (host(g2), "widened tail")):
        assert_parity(g, o.gamma, lab)
    assert r1.n_evaluated == r2.n_evaluated == o.n_evaluated
    # fixed layouts are not widened
    g3, r3 = gx.gammax_map(ref, ev, p.spacing, 0.03, 3.0, 0.1, True, tail_lanes=8, ctx=ctx)
    assert_parity(host(g3), o.gamma, "fixed 8 lanes")


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


def test_nonfinite_in_either_dose_anywhere(gx):
    """A NaN or infinity anywhere in either dose (above or below the threshold, in any prep
    tile) is refused, and the next clean map on the same context is not."""
    rng = np.random.default_rng(5)
    shape = (9, 40, 37)
    ref = (rng.uniform(0.0, 1.0, shape)).astype(np.float32)
    n = ref.size
    ctx = gx.Context(0)
    for which, idx, val in [("ref", 0, np.nan), ("ref", n - 1, np.inf), ("ev", n // 2, np.nan),
                            ("ev", n - 3, -np.inf), ("ev", 7, np.inf)]:
        r, e = ref.copy(), ref.copy()
        tgt = r if which == "ref" else e
        tgt.flat[idx] = val
        if which == "ev":
            r.flat[idx] = 0.0   # below the threshold: the node is not evaluated
        with pytest.raises(gx.GammaxError) as err:
            gx.gammax_map(dev(r), dev(e), (2.5, 2.5, 2.5), 0.03, 3.0, 0.1, ctx=ctx)
        assert err.value.status == -4, (which, idx)
        g, res = gx.gammax_map(dev(ref), dev(ref), (2.5, 2.5, 2.5), 0.03, 3.0, 0.1, ctx=ctx)
        assert res.n_evaluated == int((ref >= np.float32(0.1) * ref.max()).sum())


def test_flat_entry_point(gx):
    p = make_config_pair("2d_64x64_1mm", 4)
    a, pr = gx.gamma_map(dev(p.ref), dev(p.eval), p.spacing, 0.03, 3.0, 0.1)
    b, r = gx.gammax_map(dev(p.ref), dev(p.eval), p.spacing, 0.03, 3.0, 0.1)
    assert np.array_equal(host(a), host(b))
    assert pr == pytest.approx(r.pass_rate)


def test_steady_maps_match_timed_maps(gx):
    """Steady-state calls on the cached table, with new doses in the same buffers and eager
    work between them: each equals a timed call (events around every phase) on the same
    buffers, and the oracle."""
    import torch
    p0 = make_pair_3d(31, shape=(33, 40, 37), spacing=(2.5, 2.5, 2.5))
    ref, ev = dev(p0.ref), dev(p0.eval)
    out = torch.empty_like(ref)
    ctx = gx.Context(0)
    gx.gammax_map(ref, ev, p0.spacing, 0.03, 3.0, 0.1, out=out, ctx=ctx)      # builds the table
    for k in range(5):
        pk = make_pair_3d(40 + k, shape=(33, 40, 37), spacing=(2.5, 2.5, 2.5))
        ref.copy_(torch.from_numpy(pk.ref))
        ev.copy_(torch.from_numpy(pk.eval))
        junk = torch.randn(1 << 16, device="cuda").sum()   # unrelated eager work
        _, r_steady = gx.gammax_map(ref, ev, p0.spacing, 0.03, 3.0, 0.1, out=out, ctx=ctx)
        g_steady = host(out).copy()
        _, r_timed = gx.gammax_map(ref, ev, p0.spacing, 0.03, 3.0, 0.1, out=out, ctx=ctx, timing=True)
        assert np.array_equal(g_steady, host(out)), f"map {k}"
        assert r_steady.n_pass == r_timed.n_pass and r_steady.n_cells == r_timed.n_cells
        o = oracle.gamma(pk.ref, pk.eval, pk.spacing, 0.03, 3.0, 0.1)
        assert_parity(g_steady, o.gamma, f"map {k}")
        assert float(junk) == float(junk)
    ctx.close()


def test_radius_outgrowing_cached_table(gx):
    """A second pair with a larger search radius than the cached table covers must be
    detected on the device and redone with a larger table."""
    import torch
    ctx = gx.Context(0)
    p = make_pair_3d(50, shape=(30, 34, 32), spacing=(2.5, 2.5, 2.5))
    ref, ev = dev(p.ref), dev(p.eval)
    _, r1 = gx.gammax_map(ref, ev, p.spacing, 0.03, 3.0, 0.1, ctx=ctx)
    ev2 = ev.clone()
    ev2 += 0.2 * (ref > 0.5).float()        # large dose differences: radius grows
    o = oracle.gamma(p.ref, host(ev2), p.spacing, 0.03, 3.0, 0.1)
    g, r2 = gx.gammax_map(ref, ev2, p.spacing, 0.03, 3.0, 0.1, ctx=ctx)
    assert r2.search_radius > 1.3 * r1.search_radius
    assert r2.table_len > r1.table_len
    assert_parity(host(g), o.gamma, "grown radius")
    ctx.close()
