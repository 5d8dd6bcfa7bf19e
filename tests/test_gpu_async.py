"""GPU tests of the queued maps (gammax_map_async / gammax_map_wait): results and gamma
identical to the synchronous gammax_map of the same pair, the table build inside the
first queued call, the re-run at collection time when a radius outgrows the cached table,
dose errors reported by the wait, the slot limit, and tickets collected once.  One case
is also checked against the FP64 oracle."""
import ctypes as C

import numpy as np
import pytest

import oracle
from dosegen import make_pair_3d
from gpu_util import assert_parity, dev, host

pytestmark = pytest.mark.gpu

FIELDS = ("n_evaluated", "n_pass", "n_borderline", "n_cells", "n_tail", "n_guarded", "max_gamma", "dose_max",
          "search_radius", "table_len")


@pytest.fixture(scope="module")
def gx():
    import paper_1012_1900_amd as g
    return g


@pytest.fixture(scope="module")
def pair():
    return make_pair_3d(11, shape=(29, 36, 33), spacing=(2.5, 2.5, 2.5))


def _same(r, q):
    for f in FIELDS:
        assert getattr(r, f) == getattr(q, f), f


def test_queue_equals_sync(gx, pair):
    ref, ev = dev(pair.ref), dev(pair.eval)
    ctx = gx.Context(0)
    g1, r1 = gx.gammax_map(ref, ev, pair.spacing, 0.03, 3.0, 0.1, ctx=gx.Context(0))
    # the first queued call builds the table (runs to completion), the rest use it
    outs = [gx.gammax_map_async(ref, ev, pair.spacing, 0.03, 3.0, 0.1, ctx=ctx) for _ in range(12)]
    res = [t.wait() for t in outs]
    for t, r in zip(outs, res):
        _same(r, r1)
        assert np.array_equal(host(t.gamma), host(g1))
    # one shared output buffer, collected out of order
    out = ref.new_empty(ref.shape)
    ts = [gx.gammax_map_async(ref, ev, pair.spacing, 0.03, 3.0, 0.1, out=out, ctx=ctx) for _ in range(8)]
    for t in reversed(ts):
        _same(t.wait(), r1)
    assert np.array_equal(host(out), host(g1))
    o = oracle.gamma(pair.ref, pair.eval, pair.spacing, 0.03, 3.0, 0.1)
    assert_parity(host(out), o.gamma, "queued map")


def test_two_pairs_interleaved(gx, pair):
    other = make_pair_3d(12, shape=(29, 36, 33), spacing=(2.5, 2.5, 2.5))
    ctx = gx.Context(0)
    a = (dev(pair.ref), dev(pair.eval))
    b = (dev(other.ref), dev(other.eval))
    ga, ra = gx.gammax_map(*a, pair.spacing, 0.03, 3.0, 0.1, ctx=gx.Context(0))
    gb, rb = gx.gammax_map(*b, other.spacing, 0.03, 3.0, 0.1, ctx=gx.Context(0))
    ts = []
    for _ in range(3):
        ts.append((gx.gammax_map_async(*a, pair.spacing, 0.03, 3.0, 0.1, ctx=ctx), ga, ra))
        ts.append((gx.gammax_map_async(*b, other.spacing, 0.03, 3.0, 0.1, ctx=ctx), gb, rb))
    for t, g, r in ts:
        q = t.wait()
        assert (q.n_evaluated, q.n_pass, q.n_tail) == (r.n_evaluated, r.n_pass, r.n_tail)
        assert np.array_equal(host(t.gamma), host(g))


def test_radius_outgrows_table_rerun(gx, pair):
    ctx = gx.Context(0)
    ref, ev = dev(pair.ref), dev(pair.eval)
    gx.gammax_map_async(ref, ev, pair.spacing, 0.03, 3.0, 0.1, ctx=ctx).wait()
    # a much larger dose difference at one node: its gamma0 is far beyond the cached table
    ev2 = ev.clone()
    k = int(np.argmax(pair.ref.ravel()))
    ev2.view(-1)[k] += 0.6
    g_sync, r_sync = gx.gammax_map(ref, ev2, pair.spacing, 0.03, 3.0, 0.1, ctx=gx.Context(0))
    t = gx.gammax_map_async(ref, ev2, pair.spacing, 0.03, 3.0, 0.1, ctx=ctx)
    r = t.wait()
    _same(r, r_sync)
    assert np.array_equal(host(t.gamma), host(g_sync))
    assert r.search_radius > 5.0


def test_dose_error_reported_by_wait(gx, pair):
    ctx = gx.Context(0)
    ref, ev = dev(pair.ref), dev(pair.eval)
    gx.gammax_map_async(ref, ev, pair.spacing, 0.03, 3.0, 0.1, ctx=ctx).wait()
    bad = ev.clone()
    bad.view(-1)[17] = float("nan")
    t = gx.gammax_map_async(ref, bad, pair.spacing, 0.03, 3.0, 0.1, ctx=ctx)
    with pytest.raises(gx.GammaxError) as e:
        t.wait()
    assert e.value.status == -4
    # the context keeps working
    g, r = gx.gammax_map(ref, ev, pair.spacing, 0.03, 3.0, 0.1, ctx=ctx)
    assert r.n_evaluated > 0


def test_slot_limit_and_single_collection(gx, pair):
    from paper_1012_1900_amd import _abi
    ctx = gx.Context(0)
    ref, ev = dev(pair.ref), dev(pair.eval)
    out = ref.new_empty(ref.shape)
    gx.gammax_map_async(ref, ev, pair.spacing, 0.03, 3.0, 0.1, out=out, ctx=ctx).wait()
    ts = [gx.gammax_map_async(ref, ev, pair.spacing, 0.03, 3.0, 0.1, out=out, ctx=ctx)
          for _ in range(gx.ASYNC_SLOTS)]
    with pytest.raises(gx.GammaxError) as e:
        gx.gammax_map_async(ref, ev, pair.spacing, 0.03, 3.0, 0.1, out=out, ctx=ctx)
    assert e.value.status == -3
    first = ts[0].wait()
    # a collected ticket is unknown to the library from then on
    lib = _abi.raw_library()
    r = _abi.Result()
    assert lib.gammax_map_wait(ctx.handle, ts[0].ticket, C.byref(r)) == _abi.E_PARAM
    assert lib.gammax_map_wait(ctx.handle, 0, C.byref(r)) == _abi.E_PARAM
    for t in ts[1:]:
        _same(t.wait(), first)
    # timing is refused for queued maps
    p = _abi.make_problem(tuple(ref.shape), pair.spacing, 0.03, 3.0, 0.1, False)
    o = _abi.make_options("none", "guarded", 1e6, True, 0, 0, "plain", None, 1.1)
    tk = C.c_uint64(5)
    st = lib.gammax_map_async(ctx.handle, C.byref(p), C.byref(o), ref.data_ptr(), ev.data_ptr(), out.data_ptr(),
                              C.byref(tk), None)
    assert st == _abi.E_PARAM and tk.value == 0


def test_queued_learned_and_2d(gx, pair):
    """Queued maps with the learned radius (the network among the queued launches) and of a
    2D pair: the same gamma and counts as the synchronous calls."""
    from dosegen import make_config_pair
    from oracle import cnn
    model = gx.Model(cnn.init_params(5).astype(np.float32))
    ref, ev = dev(pair.ref), dev(pair.eval)
    kw = dict(radius="learned", sort="predicted", model=model)
    g1, r1 = gx.gammax_map(ref, ev, pair.spacing, 0.03, 3.0, 0.1, ctx=gx.Context(0), **kw)
    ctx = gx.Context(0)
    ts = [gx.gammax_map_async(ref, ev, pair.spacing, 0.03, 3.0, 0.1, ctx=ctx, **kw) for _ in range(4)]
    for t in ts:
        r = t.wait()
        _same(r, r1)
        assert r.n_fallback == r1.n_fallback
        assert np.array_equal(host(t.gamma), host(g1))
    p2 = make_config_pair("2d_64x64_1mm", 3)
    a, b = dev(p2.ref), dev(p2.eval)
    g2, r2 = gx.gammax_map(a, b, p2.spacing, 0.03, 3.0, 0.1, ctx=gx.Context(0))
    ctx2 = gx.Context(0)
    ts = [gx.gammax_map_async(a, b, p2.spacing, 0.03, 3.0, 0.1, ctx=ctx2) for _ in range(3)]
    for t in ts:
        _same(t.wait(), r2)
        assert np.array_equal(host(t.gamma), host(g2))
