"""GPU gamma maps against the FP64 oracle at the sizes the targets are stated on.

* 128x128x96 at 2.5 mm (the benchmark workload) at 3%/3mm, 2%/2mm and 1%/1mm: every node;
* 256x256x192 at 1.25 mm at 3%/3mm and 2%/2mm, plain and with the learned radius (the
  shipped network on the 2x pooled input, the benchmark's learned leg): every node;
* the same grid at 1%/3mm, the costliest point of the criteria study: every node;
* the FP32 / guarded / FP64 projection ablation of that grid: per-node error against the
  oracle;
* the extreme points of the scaling studies, on sampled nodes (random plus the largest
  gamma0): the dose shift of -10 % and +10 % inside the 10 % region, and the 72x512x512
  grid of the resolution study.

Every masked node must lie within |dgamma| <= 1e-5 + 1e-5 gamma of the oracle, with the
same mask and the same pass decisions outside the 1e-5 band around gamma = 1.
"""
import os

import numpy as np
import pytest

import oracle
from dosegen import make_config_pair, make_pair_3d
from gpu_util import assert_parity, dev, host

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_1012_1900_amd", "weights", "cnn_3d_2.5mm_3pct3mm.npy")


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def gx():
    import paper_1012_1900_amd as g
    return g


@pytest.fixture(scope="module")
def c1():
    return make_config_pair("3d_128x128x96_2.5mm", 100)


@pytest.fixture(scope="module")
def c2():
    return make_config_pair("3d_256x256x192_1.25mm", 200)


def _counts_agree(r, o):
    assert r.n_evaluated == o.n_evaluated
    assert abs(int(r.n_pass) - o.n_pass) <= o.n_borderline + r.n_borderline


@pytest.mark.parametrize("crit", [(0.03, 3.0), (0.02, 2.0), (0.01, 1.0)])
def test_c1_every_node(gx, c1, crit):
    p = c1
    _say(f"128x128x96 {crit}")
    o = oracle.gamma(p.ref, p.eval, p.spacing, *crit, 0.1)
    g, r = gx.gammax_map(dev(p.ref), dev(p.eval), p.spacing, *crit, 0.1)
    assert_parity(host(g), o.gamma, f"128x128x96 {crit}")
    _counts_agree(r, o)
    assert o.cells_visited * (1 - 1e-4) <= r.n_cells <= o.cells_visited + 63 * r.n_tail


@pytest.mark.parametrize("crit", [(0.03, 3.0), (0.02, 2.0), (0.01, 3.0)])
def test_c2_every_node(gx, c2, crit):
    p = c2
    _say(f"256x256x192 {crit}")
    o = oracle.gamma(p.ref, p.eval, p.spacing, *crit, 0.1)
    g, r = gx.gammax_map(dev(p.ref), dev(p.eval), p.spacing, *crit, 0.1)
    assert_parity(host(g), o.gamma, f"256x256x192 {crit}")
    _counts_agree(r, o)


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="trained weights not present")
@pytest.mark.parametrize("crit", [(0.03, 3.0), (0.02, 2.0)])
def test_c2_learned_every_node(gx, c2, crit):
    """The learned radius with the shipped network on the pooled input (as the benchmark
    runs it): bit for bit the plain map, and within the bar of the oracle."""
    p = c2
    _say(f"256x256x192 learned {crit}")
    ref, ev = dev(p.ref), dev(p.eval)
    model = gx.Model(np.load(WEIGHTS, allow_pickle=False))
    g_plain, r_plain = gx.gammax_map(ref, ev, p.spacing, *crit, 0.1)
    g, r = gx.gammax_map(ref, ev, p.spacing, *crit, 0.1, radius="learned", sort="predicted", model=model,
                         cnn_pool=2)
    assert np.array_equal(host(g), host(g_plain))
    assert (r.n_pass, r.n_borderline, r.n_tail) == (r_plain.n_pass, r_plain.n_borderline, r_plain.n_tail)
    assert r.n_tail > 0 and r.n_fallback <= r.n_tail
    o = oracle.gamma(p.ref, p.eval, p.spacing, *crit, 0.1)
    assert_parity(host(g), o.gamma, f"256x256x192 learned {crit}")
    _counts_agree(r, o)
    # visited cells: the exact walk's, plus at most lanes - 1 rows past the break per tail
    # node (the lane groups evaluate rows in batches)
    for rr in (r, r_plain):
        assert o.cells_visited * (1 - 1e-4) <= rr.n_cells <= o.cells_visited + 63 * rr.n_tail


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="trained weights not present")
def test_c2_learned_short_and_long_tail_forms(gx, c2):
    """A fresh context knows no tail yet, so its first learned map takes the short-tail form
    (groups of 64 lanes walk with the plain bound; the nodes the prediction would not have
    certified are counted); the next map, knowing the tail is long, takes the speculative
    walk and its fallback list.  Both are the plain map bit for bit and count the same
    fallbacks."""
    p = c2
    _say("256x256x192 learned: short-tail form, then the fallback list")
    ref, ev = dev(p.ref), dev(p.eval)
    model = gx.Model(np.load(WEIGHTS, allow_pickle=False))
    g_plain, r_plain = gx.gammax_map(ref, ev, p.spacing, 0.03, 3.0, 0.1)
    assert r_plain.n_tail > 4096
    ctx = gx.Context(0)
    kw = dict(radius="learned", sort="predicted", model=model, cnn_pool=2, ctx=ctx)
    g1, r1 = gx.gammax_map(ref, ev, p.spacing, 0.03, 3.0, 0.1, **kw)
    g2, r2 = gx.gammax_map(ref, ev, p.spacing, 0.03, 3.0, 0.1, **kw)
    for g, r in ((g1, r1), (g2, r2)):
        assert np.array_equal(host(g), host(g_plain))
        assert (r.n_pass, r.n_tail) == (r_plain.n_pass, r_plain.n_tail)
    assert 0 < r1.n_fallback == r2.n_fallback < r1.n_tail


def test_c2_precision_ablation(gx, c2):
    """FP32 projections everywhere, the FP64 guard of ill-conditioned tetrahedra, and FP64
    everywhere: each within the bar at every node; FP64 within float rounding of the
    oracle."""
    p = c2
    _say("256x256x192 precision ablation")
    o = oracle.gamma(p.ref, p.eval, p.spacing, 0.03, 3.0, 0.1)
    m = o.gamma >= 0
    err = {}
    for prec in ("fp32", "guarded", "fp64"):
        g, r = gx.gammax_map(dev(p.ref), dev(p.eval), p.spacing, 0.03, 3.0, 0.1, precision=prec)
        err[prec] = assert_parity(host(g), o.gamma, f"256x256x192 {prec}")
        _counts_agree(r, o)
        if prec == "fp64":
            gh = host(g).astype(np.float64)
            assert np.all(np.abs(gh[m] - o.gamma[m]) <= 1e-7 * np.maximum(1.0, o.gamma[m]))
    _say(f"max |dgamma|: {err}")
    assert err["fp64"] <= err["fp32"] + 1e-12


def _sampled(p, g, crit, label, n=3000, heavy=300, seed=5):
    gh = host(g).ravel()
    masked = np.flatnonzero(gh >= 0)
    rng = np.random.default_rng(seed)
    g0 = np.abs(p.eval.ravel()[masked].astype(np.float64) - p.ref.ravel()[masked])
    idx = np.unique(np.concatenate([rng.choice(masked, min(n, masked.size), replace=False),
                                    masked[np.argsort(g0)[-heavy:]]]))
    o = oracle.gamma(p.ref, p.eval, p.spacing, *crit, 0.1, subset=idx)
    assert_parity(gh[idx], o.gamma, label)
    return o


class _Shifted:
    def __init__(self, p, s):
        dmax = float(p.ref.max())
        region = p.ref >= np.float32(0.1) * np.float32(dmax)
        self.ref = p.ref
        self.eval = np.where(region, p.eval + np.float32(s * dmax), p.eval).astype(np.float32)
        self.spacing = p.spacing


@pytest.mark.parametrize("shift", [-0.10, 0.10])
def test_c2_dose_shift_extremes_sampled(gx, c2, shift):
    """The dose-shift study's extreme points (evaluation dose + s Dmax inside the 10 %
    region): most nodes walk far past the key-0 cells."""
    p = _Shifted(c2, shift)
    _say(f"256x256x192 shift {shift}")
    g, r = gx.gammax_map(dev(p.ref), dev(p.eval), p.spacing, 0.03, 3.0, 0.1)
    assert r.n_tail > 10 ** 6
    o = _sampled(p, g, (0.03, 3.0), f"shift {shift}")
    assert r.n_evaluated == o.n_masked


def test_resolution_extreme_sampled(gx):
    """The resolution study's largest grid: 72x512x512 over the 240x320x320 mm box."""
    shape = (72, 512, 512)
    spacing = tuple(b / n for b, n in zip((240.0, 320.0, 320.0), shape))
    _say("72x512x512")
    p = make_pair_3d(200, shape=shape, spacing=spacing)
    g, r = gx.gammax_map(dev(p.ref), dev(p.eval), p.spacing, 0.03, 3.0, 0.1)
    o = _sampled(p, g, (0.03, 3.0), "72x512x512")
    assert r.n_evaluated == o.n_masked
