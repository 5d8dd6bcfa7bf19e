"""GPU tests of the queued per-pair maps (gammax_map_many) beside the graph batch
(gammax_batch): every pair's gamma and counts are the same through both and through the
single map, one case matches the FP64 oracle, repeated calls give the same maps, and an
error names its pair."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_parity, dev, host

pytestmark = pytest.mark.gpu

FIELDS = ("n_evaluated", "n_pass", "n_borderline", "n_cells", "n_tail", "n_guarded", "max_gamma",
          "search_radius", "table_len")


@pytest.fixture(scope="module")
def gx():
    import paper_1012_1900_amd as g
    return g


@pytest.fixture(scope="module")
def pairs():
    from dosegen import batch_specs, make_batch_pair
    out = []
    for sp in batch_specs(42000, 9, 0.2):
        p = make_batch_pair(sp)
        out.append(dict(ref=dev(p.ref), ev=dev(p.eval), spacing=p.spacing, dd=sp.dd, dta=sp.dta, local=sp.local,
                        host=p))
    return out


def test_batch_equals_many_and_single(gx, pairs):
    ctx = gx.Context(0)
    gb, rb = gx.gammax_batch(pairs, ctx=ctx)
    gm, rm = gx.gammax_map_many(pairs, ctx=gx.Context(0))
    for i, q in enumerate(pairs):
        assert np.array_equal(host(gb[i]), host(gm[i])), i
        g1, r1 = gx.gammax_map(q["ref"], q["ev"], q["spacing"], q["dd"], q["dta"], 0.1, q["local"],
                               ctx=gx.Context(0))
        assert np.array_equal(host(gb[i]), host(g1)), i
        for f in FIELDS:
            assert getattr(rb[i], f) == getattr(rm[i], f) == getattr(r1, f), (i, f)
        assert np.isfinite(rb[i].ms_done) and rb[i].ms_done > 0.0, (i, rb[i].ms_done)
    # repeated calls on the cached per-pair contexts
    gb2, rb2 = gx.gammax_batch(pairs, ctx=ctx)
    gm2, _ = gx.gammax_map_many(pairs, ctx=gx.Context(0))
    for a, b, m2 in zip(gb, gb2, gm2):
        assert np.array_equal(host(a), host(b)) and np.array_equal(host(a), host(m2))
    q = pairs[1]
    p = q["host"]
    o = oracle.gamma(p.ref, p.eval, p.spacing, q["dd"], q["dta"], 0.1, q["local"])
    assert_parity(host(gb[1]), o.gamma, "batch pair 1")


def test_batch_error_names_the_pair(gx, pairs):
    bad = [dict(q) for q in pairs[:3]]
    ev = bad[1]["ev"].clone()
    ev.view(-1)[5] = float("inf")
    bad[1]["ev"] = ev
    ctx = gx.Context(0)
    with pytest.raises(gx.GammaxError) as e:
        gx.gammax_map_many(bad, ctx=ctx)
    assert e.value.status == -4 and "pair 1" in str(e.value)
    gs, rs = gx.gammax_map_many(pairs[:3], ctx=ctx)
    assert all(r.n_evaluated > 0 for r in rs)
