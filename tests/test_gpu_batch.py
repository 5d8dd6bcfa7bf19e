"""GPU tests of gammax_batch: a mixed batch (2D and 3D, sizes, spacings, criteria, global
and local) returns for every pair exactly what gammax_map returns for it alone, and what
the FP64 oracle returns, through graph replays, autotuning, the learned radius, the FP64
guard and a radius that outgrows a pair's cached table."""
import numpy as np
import pytest

from gpu_util import assert_parity, dev, host

# Written for the first batch pipeline (a persistent key-0 kernel striding over the items
# and atomic work queues for the tail phases), whose first GPU run stopped making progress
# with the cause never found.  That pipeline is removed; gammax_batch is now one captured
# graph of the single-map kernels and one key-0 launch over all pairs, tested in
# test_gpu_batch_graph.py.  These stay skipped.
pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="tests of the removed persistent batch pipeline, whose first GPU run did not "
                                      "finish (cause not found); the graph batch is tested in test_gpu_batch_graph.py")]


@pytest.fixture(scope="module")
def gx():
    import paper_1012_1900_amd as g
    return g


def _specs(seed=40000, n=10, scale=0.16):
    from dosegen import batch_specs
    return batch_specs(seed, n, scale)


@pytest.fixture(scope="module")
def batch():
    from dosegen import make_batch_pair
    out = []
    for sp in _specs():
        p = make_batch_pair(sp)
        out.append(dict(ref=dev(p.ref), ev=dev(p.eval), spacing=p.spacing, dd=sp.dd, dta=sp.dta,
                        local=sp.local, host=p))
    return out


def _singles(gx, pairs, **kw):
    outs = []
    for q in pairs:
        g, r = gx.gammax_map(q["ref"], q["ev"], q["spacing"], q["dd"], q["dta"], 0.1, q["local"], **kw)
        outs.append((host(g), r))
    return outs


def test_batch_equals_single_maps(gx, batch):
    kinds = {q["ref"].dim() for q in batch}
    assert kinds == {2, 3} and any(q["local"] for q in batch) and not all(q["local"] for q in batch)
    ctx = gx.Context(0)
    gs, rs = gx.gammax_batch(batch, ctx=ctx)
    single = _singles(gx, batch)
    for i, ((g1, r1), g, r) in enumerate(zip(single, gs, rs)):
        assert np.array_equal(host(g), g1), i
        assert (r.n_evaluated, r.n_pass, r.n_borderline, r.n_tail) == (r1.n_evaluated, r1.n_pass, r1.n_borderline,
                                                                      r1.n_tail), i
        assert r.ms_done > 0.0
    # replays of the captured batch
    for _ in range(2):
        gs2, _ = gx.gammax_batch(batch, ctx=ctx)
        for a, b in zip(gs, gs2):
            assert np.array_equal(host(a), host(b))


def test_batch_matches_oracle(gx, batch):
    import oracle
    gs, _ = gx.gammax_batch(batch)
    for i in (0, 3, 7):
        q = batch[i]
        p = q["host"]
        o = oracle.gamma(p.ref, p.eval, p.spacing, q["dd"], q["dta"], 0.1, q["local"])
        assert_parity(host(gs[i]), o.gamma, f"batch pair {i}")


def test_batch_autotune_and_tuning_file(gx, batch, tmp_path):
    ctx = gx.Context(0)
    ref, _ = gx.gammax_batch(batch, ctx=ctx)
    gs, _ = gx.gammax_batch(batch, ctx=ctx, autotune=True)
    for a, b in zip(ref, gs):
        assert np.array_equal(host(a), host(b))
    path = str(tmp_path / "tune.txt")
    gx.tune_save(path, ctx)
    lines = open(path).read().split()
    assert len(lines) >= 2 and all(int(v) in (0, 8, 16, 32, 64) for v in lines[1::2])
    ctx2 = gx.Context(0)
    gx.tune_load(path, ctx2)
    gs2, _ = gx.gammax_batch(batch, ctx=ctx2, autotune=True)
    for a, b in zip(ref, gs2):
        assert np.array_equal(host(a), host(b))


@pytest.mark.parametrize("lanes", [1, 8, 64])
def test_batch_fixed_tail_layouts(gx, batch, lanes):
    ref, _ = gx.gammax_batch(batch)
    gs, _ = gx.gammax_batch(batch, tail_lanes=lanes)
    for a, b in zip(ref, gs):
        assert np.array_equal(host(a), host(b))


def test_batch_learned_and_guard(gx, batch):
    from oracle import cnn
    m = gx.Model(cnn.init_params(3).astype(np.float32))
    ref, _ = gx.gammax_batch(batch)
    gs, rs = gx.gammax_batch(batch, radius="learned", model=m)
    for a, b in zip(ref, gs):
        assert np.array_equal(host(a), host(b))
    assert sum(r.n_fallback for r in rs) > 0
    single = _singles(gx, batch, cond_threshold=1.0)
    gs, rs = gx.gammax_batch(batch, cond_threshold=1.0)
    for (g1, r1), g, r in zip(single, gs, rs):
        assert np.array_equal(host(g), g1)
    assert sum(r.n_guarded for r in rs) > 0


def test_batch_radius_outgrows_table(gx, batch):
    import torch
    ctx = gx.Context(0)
    gx.gammax_batch(batch, ctx=ctx)
    # a larger dose difference in one pair: its radius outgrows its cached table
    bigger = [dict(q) for q in batch]
    k = next(i for i, q in enumerate(batch) if q["ref"].dim() == 3)
    ev = bigger[k]["ev"].clone()
    flat = ev.view(-1)
    flat[flat.numel() // 2] += 0.5
    bigger[k]["ev"] = ev
    gs, _ = gx.gammax_batch(bigger, ctx=ctx)
    single = _singles(gx, bigger)
    for (g1, _), g in zip(single, gs):
        assert np.array_equal(host(g), g1)
    torch.cuda.synchronize()


def test_batch_errors(gx, batch):
    bad = [dict(q) for q in batch[:3]]
    ev = bad[1]["ev"].clone()
    ev.view(-1)[5] = float("nan")
    bad[1]["ev"] = ev
    with pytest.raises(gx.GammaxError) as e:
        gx.gammax_batch(bad)
    assert e.value.status == -4 and "pair 1" in str(e.value)
