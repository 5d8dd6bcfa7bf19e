"""GPU tests of gammax_map_noalloc, the map whose workspace is the library's fixed device
array: its gamma and counts equal those of gammax_map (the context entry point) bit for bit,
and the FP64 oracle's within the parity bar, on two calls in a row (the second on a smaller
grid, so the array holds the larger call's contents when it starts), in 3D and 2D, with the
sort and precision options; sizes beyond its limits are refused before any launch."""
import numpy as np
import pytest

import oracle
from dosegen import make_config_pair, make_pair_3d
from gpu_util import assert_parity, dev, host

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def gx():
    import paper_1012_1900_amd as g
    return g


def _both(gx, p, dd, dta, local=False, **kw):
    import torch
    ref, ev = dev(p.ref), dev(p.eval)
    out = torch.full_like(ref, 7.0)   # stale values: every node must be written
    r_na = gx.gammax_map_noalloc(ref, ev, p.spacing, dd, dta, 0.1, local, out=out, **kw)
    torch.cuda.synchronize()
    g_ctx, r_ctx = gx.gammax_map(ref, ev, p.spacing, dd, dta, 0.1, local, ctx=gx.Context(0), **kw)
    return host(out), r_na, host(g_ctx), r_ctx


def _same(g_na, r_na, g_ctx, r_ctx, label):
    assert np.array_equal(g_na.view(np.uint32), g_ctx.view(np.uint32)), label
    for f in ("n_evaluated", "n_pass", "n_borderline", "n_fp64_tets", "n_cells", "n_tail", "n_guarded"):
        assert getattr(r_na, f) == getattr(r_ctx, f), (label, f)
    assert r_na.max_gamma == r_ctx.max_gamma and r_na.search_radius == r_ctx.search_radius, label


def test_two_calls_larger_then_smaller(gx):
    big = make_config_pair("3d_128x128x96_2.5mm", 100)
    small = make_pair_3d(7, shape=(40, 48, 56), spacing=(2.5, 2.0, 3.0))
    for label, p, crit in (("128x128x96 3%/3mm", big, (0.03, 3.0)), ("40x48x56 2%/2mm", small, (0.02, 2.0))):
        _say(f"noalloc {label}")
        g_na, r_na, g_ctx, r_ctx = _both(gx, p, *crit)
        _same(g_na, r_na, g_ctx, r_ctx, label)
        o = oracle.gamma(p.ref, p.eval, p.spacing, *crit, 0.1)
        assert_parity(g_na, o.gamma, label)
        assert r_na.n_evaluated == o.n_evaluated
        assert 0 < r_na.table_len <= gx.NOALLOC_MAX_TABLE


def test_2d_local_and_options(gx):
    p2 = make_config_pair("2d_64x64_1mm", 3)
    p3 = make_pair_3d(11, shape=(24, 32, 40), spacing=(2.5, 2.5, 2.5))
    cases = [("2d global", p2, False, {}), ("2d local", p2, True, {}),
             ("3d dd sort", p3, False, {"sort": "dd"}), ("3d bound sort 8 lanes", p3, False, {"sort": "bound", "tail_lanes": 8}),
             ("3d fp32", p3, False, {"precision": "fp32"}), ("3d fp64", p3, False, {"precision": "fp64"}),
             ("3d local", p3, True, {})]
    for label, p, local, kw in cases:
        _say(f"noalloc {label}")
        g_na, r_na, g_ctx, r_ctx = _both(gx, p, 0.03, 3.0, local, **kw)
        _same(g_na, r_na, g_ctx, r_ctx, label)
        o = oracle.gamma(p.ref, p.eval, p.spacing, 0.03, 3.0, 0.1, local)
        assert_parity(g_na, o.gamma, label)


def test_limits_and_refusals(gx):
    import torch
    # more nodes than the array holds: refused on the host, before any launch
    n = 2 * 1024 * 1032
    ref = torch.zeros((2, 1024, 1032), dtype=torch.float32, device="cuda")
    assert ref.numel() == n > gx.NOALLOC_MAX_NODES
    ev = torch.zeros_like(ref)
    out = torch.empty_like(ref)
    with pytest.raises(gx.GammaxError) as e:
        gx.gammax_map_noalloc(ref, ev, (1.0, 1.0, 1.0), 0.03, 3.0, 0.1, out=out)
    assert e.value.status == -2
    # a non-finite dose is reported, and a later call still works
    p = make_pair_3d(5, shape=(16, 20, 24), spacing=(2.5, 2.5, 2.5))
    bad = p.eval.copy()
    bad[3, 4, 5] = np.nan
    r, b = dev(p.ref), dev(bad)
    out = torch.empty_like(r)
    with pytest.raises(gx.GammaxError) as e:
        gx.gammax_map_noalloc(r, b, p.spacing, 0.03, 3.0, 0.1, out=out)
    assert e.value.status == -4
    res = gx.gammax_map_noalloc(r, dev(p.eval), p.spacing, 0.03, 3.0, 0.1, out=out)
    o = oracle.gamma(p.ref, p.eval, p.spacing, 0.03, 3.0, 0.1)
    assert_parity(host(out), o.gamma, "after an error")
    assert res.n_evaluated == o.n_evaluated
