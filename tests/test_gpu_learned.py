"""GPU tests of the learned search radius: the speculative walk inside f * gamma_hat with
its fallback returns exactly the plain search's gamma, whatever the prediction (a random
network, one that predicts 0 everywhere so that every tail node falls back, one that
predicts a huge radius so that none does), in every tail layout and order."""
import os

import numpy as np
import pytest

from gpu_util import assert_parity, dev, host

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_1012_1900_amd", "weights", "cnn_3d_2.5mm_3pct3mm.npy")


@pytest.fixture(scope="module")
def gx():
    import paper_1012_1900_amd as g
    return g


def _params(kind):
    from oracle import cnn
    if kind == "random":
        return cnn.init_params(21).astype(np.float32)
    th = np.zeros(cnn.n_params(), dtype=np.float32)
    # only the last bias: y = b everywhere
    th[-1] = np.log(0.01) if kind == "zero" else 10.0
    return th


@pytest.fixture(scope="module")
def models(gx):
    return {k: gx.Model(_params(k)) for k in ("random", "zero", "huge")}


@pytest.fixture(scope="module")
def pair():
    from dosegen import make_pair_3d
    return make_pair_3d(31, shape=(40, 48, 56), spacing=(2.5, 2.5, 2.5))


@pytest.mark.parametrize("kind", ["random", "zero", "huge"])
@pytest.mark.parametrize("tail_lanes", [0, 1, 16])
@pytest.mark.parametrize("sort", ["none", "predicted"])
@pytest.mark.parametrize("crit", [(0.03, 3.0), (0.01, 1.0)])
def test_learned_equals_plain(gx, models, pair, kind, tail_lanes, sort, crit):
    dd, dta = crit
    ref, ev = dev(pair.ref), dev(pair.eval)
    g_plain, r_plain = gx.gammax_map(ref, ev, pair.spacing, dd, dta, 0.1, tail_lanes=tail_lanes)
    g_l, r_l = gx.gammax_map(ref, ev, pair.spacing, dd, dta, 0.1, tail_lanes=tail_lanes,
                             radius="learned", sort=sort, model=models[kind])
    assert np.array_equal(host(g_plain), host(g_l))
    assert (r_l.n_pass, r_l.n_borderline, r_l.n_tail) == (r_plain.n_pass, r_plain.n_borderline, r_plain.n_tail)
    assert r_plain.n_tail > 0
    if kind == "zero":
        assert r_l.n_fallback == r_l.n_tail
    elif kind == "huge":
        assert r_l.n_fallback == 0


def test_predicted_order_alone(gx, models, pair):
    ref, ev = dev(pair.ref), dev(pair.eval)
    g_plain, _ = gx.gammax_map(ref, ev, pair.spacing, 0.02, 2.0, 0.1)
    g_l, r_l = gx.gammax_map(ref, ev, pair.spacing, 0.02, 2.0, 0.1, sort="predicted", model=models["random"])
    assert np.array_equal(host(g_plain), host(g_l))
    assert r_l.n_fallback == 0


def test_learned_matches_oracle(gx, models, pair):
    import oracle
    ref, ev = dev(pair.ref), dev(pair.eval)
    g, _ = gx.gammax_map(ref, ev, pair.spacing, 0.02, 2.0, 0.1, radius="learned", sort="predicted",
                         model=models["random"])
    o = oracle.gamma(pair.ref, pair.eval, pair.spacing, 0.02, 2.0, 0.1)
    assert_parity(host(g), o.gamma, "learned 2%/2mm")


def test_learned_with_forced_guard(gx, models, pair):
    ref, ev = dev(pair.ref), dev(pair.eval)
    kw = dict(cond_threshold=1.0, tail_lanes=1)
    g_plain, r_p = gx.gammax_map(ref, ev, pair.spacing, 0.03, 3.0, 0.1, **kw)
    g_l, r_l = gx.gammax_map(ref, ev, pair.spacing, 0.03, 3.0, 0.1, radius="learned", model=models["zero"], **kw)
    assert r_p.n_guarded > 0
    assert np.array_equal(host(g_plain), host(g_l))


def test_learned_replays_and_timing(gx, models, pair):
    ref, ev = dev(pair.ref), dev(pair.eval)
    kw = dict(radius="learned", sort="predicted", model=models["random"])
    first, _ = gx.gammax_map(ref, ev, pair.spacing, 0.03, 3.0, 0.1, **kw)
    first = host(first)
    for _ in range(3):
        g, _ = gx.gammax_map(ref, ev, pair.spacing, 0.03, 3.0, 0.1, **kw)
        assert np.array_equal(host(g), first)
    _, r = gx.gammax_map(ref, ev, pair.spacing, 0.03, 3.0, 0.1, timing=True, **kw)
    assert r.ms_cnn > 0.0
    _, r = gx.gammax_map(ref, ev, pair.spacing, 0.03, 3.0, 0.1, timing=True)
    assert r.ms_cnn == 0.0


def test_learned_in_2d_is_the_plain_search(gx, models):
    from dosegen import make_pair_2d
    p = make_pair_2d(5)
    ref, ev = dev(p.ref), dev(p.eval)
    g_plain, _ = gx.gammax_map(ref, ev, p.spacing, 0.03, 3.0, 0.1)
    g_l, r = gx.gammax_map(ref, ev, p.spacing, 0.03, 3.0, 0.1, radius="learned", sort="predicted",
                           model=models["zero"])
    assert np.array_equal(host(g_plain), host(g_l))
    assert r.n_fallback == 0


def test_learned_needs_a_model(gx, pair):
    ref, ev = dev(pair.ref), dev(pair.eval)
    with pytest.raises(gx.GammaxError) as e:
        gx.gammax_map(ref, ev, pair.spacing, 0.03, 3.0, 0.1, radius="learned")
    assert e.value.status == -1
    with pytest.raises(gx.GammaxError):
        gx.gammax_map(ref, ev, pair.spacing, 0.03, 3.0, 0.1, radius="learned", model=None, radius_factor=0.5)
