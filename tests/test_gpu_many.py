"""GPU tests of gammax_map_many: a mixed set of pairs (2D and 3D, sizes, spacings, criteria,
global and local) returns for every pair exactly what gammax_map returns for it alone,
and matches the FP64 oracle; repeated calls (graph replays on the cached per-pair
contexts) give the same maps; the learned radius; an error names its pair."""
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
    for sp in batch_specs(41000, 12, 0.2):
        p = make_batch_pair(sp)
        out.append(dict(ref=dev(p.ref), ev=dev(p.eval), spacing=p.spacing, dd=sp.dd, dta=sp.dta, local=sp.local,
                        host=p))
    return out


def _single(gx, q, **kw):
    g, r = gx.gammax_map(q["ref"], q["ev"], q["spacing"], q["dd"], q["dta"], 0.1, q["local"],
                         ctx=gx.Context(0), **kw)
    return host(g), r


def test_many_equals_single_maps(gx, pairs):
    assert {q["ref"].dim() for q in pairs} == {2, 3}
    assert any(q["local"] for q in pairs) and not all(q["local"] for q in pairs)
    ctx = gx.Context(0)
    gs, rs = gx.gammax_map_many(pairs, ctx=ctx)
    for i, (q, g, r) in enumerate(zip(pairs, gs, rs)):
        g1, r1 = _single(gx, q)
        assert np.array_equal(host(g), g1), i
        for f in FIELDS:
            assert getattr(r, f) == getattr(r1, f), (i, f)
    # replays on the cached contexts
    for _ in range(2):
        gs2, rs2 = gx.gammax_map_many(pairs, ctx=ctx)
        for a, b in zip(gs, gs2):
            assert np.array_equal(host(a), host(b))
    for i in (0, 3, 7):
        q = pairs[i]
        p = q["host"]
        o = oracle.gamma(p.ref, p.eval, p.spacing, q["dd"], q["dta"], 0.1, q["local"])
        assert_parity(host(gs[i]), o.gamma, f"pair {i}")


def test_many_learned_radius(gx, pairs):
    from oracle import cnn
    model = gx.Model(cnn.init_params(7).astype(np.float32))
    three = [q for q in pairs if q["ref"].dim() == 3]
    plain, _ = gx.gammax_map_many(three, ctx=gx.Context(0))
    gs, rs = gx.gammax_map_many(three, radius="learned", sort="predicted", model=model, ctx=gx.Context(0))
    for a, b in zip(plain, gs):
        assert np.array_equal(host(a), host(b))


def test_many_error_names_the_pair(gx, pairs):
    bad = [dict(q) for q in pairs[:4]]
    ev = bad[2]["ev"].clone()
    ev.view(-1)[3] = float("nan")
    bad[2]["ev"] = ev
    ctx = gx.Context(0)
    with pytest.raises(gx.GammaxError) as e:
        gx.gammax_map_many(bad, ctx=ctx)
    assert e.value.status == -4 and "pair 2" in str(e.value)
    # the context keeps working
    gs, rs = gx.gammax_map_many(pairs[:4], ctx=ctx)
    assert all(r.n_evaluated > 0 for r in rs)
