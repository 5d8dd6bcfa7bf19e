"""Pins of the CNN oracle (learned search radius) against library routines, closed forms,
finite differences and invariants.  CPU only."""
import numpy as np
import pytest
import scipy.signal
import torch

from oracle import cnn


def _rand_theta(seed, scale=1.0):
    th = cnn.init_params(seed) * scale
    rng = np.random.default_rng(seed + 1)
    # non-zero biases so the bias paths are exercised
    k = 0
    for ws, bs in cnn.layer_shapes():
        k += int(np.prod(ws))
        th[k:k + bs[0]] = rng.uniform(-0.2, 0.2, bs[0])
        k += bs[0]
    return th


def test_param_count():
    # 2*16*27+16 + 2*(16*16*27+16) + 16*27+1
    assert cnn.n_params() == 15169
    th = _rand_theta(3)
    assert np.array_equal(cnn.flatten(cnn.unflatten(th)), th)


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(3, 7, 6, 9))
    w = rng.normal(size=(4, 3, 3, 3, 3))
    b = rng.normal(size=4)
    out = cnn.conv3d_valid(x, w, b)
    for o in range(4):
        ref = sum(scipy.signal.correlate(x[i], w[o, i], mode="valid") for i in range(3)) + b[o]
        np.testing.assert_allclose(out[o], ref, rtol=1e-12, atol=1e-12)


def test_conv_delta_kernel_is_a_shift():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(1, 6, 5, 7))
    for dz, dy, dx in [(0, 0, 0), (2, 1, 0), (1, 2, 2)]:
        w = np.zeros((1, 1, 3, 3, 3))
        w[0, 0, dz, dy, dx] = 1.0
        out = cnn.conv3d_valid(x, w, np.zeros(1))
        np.testing.assert_array_equal(out[0], x[0, dz:dz + 4, dy:dy + 3, dx:dx + 5])


def test_bwd_data_is_the_adjoint():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(3, 6, 7, 5))
    w = rng.normal(size=(4, 3, 3, 3, 3))
    g = rng.normal(size=(4, 4, 5, 3))
    lhs = np.sum(cnn.conv3d_valid(x, w, np.zeros(4)) * g)
    rhs = np.sum(x * cnn.conv3d_bwd_data(g, w, x.shape[1:]))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def test_bwd_weight_by_finite_differences():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(2, 5, 6, 5))
    w = rng.normal(size=(3, 2, 3, 3, 3))
    b = rng.normal(size=3)
    g = rng.normal(size=(3, 3, 4, 3))
    gw, gb = cnn.conv3d_bwd_weight(x, g)
    f = lambda w_, b_: np.sum(cnn.conv3d_valid(x, w_, b_) * g)  # noqa: E731
    h = 1e-6
    for idx in [(0, 0, 0, 0, 0), (2, 1, 2, 1, 0), (1, 0, 1, 2, 2)]:
        wp, wm = w.copy(), w.copy()
        wp[idx] += h
        wm[idx] -= h
        assert abs((f(wp, b) - f(wm, b)) / (2 * h) - gw[idx]) < 1e-6 * max(1, abs(gw[idx]))
    for o in range(3):
        bp, bm = b.copy(), b.copy()
        bp[o] += h
        bm[o] -= h
        assert abs((f(w, bp) - f(w, bm)) / (2 * h) - gb[o]) < 1e-6 * max(1, abs(gb[o]))


def _tiny_case(seed, shape=(7, 6, 8)):
    rng = np.random.default_rng(seed)
    feats = rng.normal(size=(2,) + shape)
    gamma = np.exp(rng.normal(size=shape) * 0.5) * 0.3
    mask = rng.uniform(size=shape) < 0.7
    gamma = np.where(mask, gamma, -1.0)
    return feats, gamma, mask


def test_network_gradient_by_finite_differences():
    """Exact (unrounded) network: every layer's weights and biases, ReLU backward, loss."""
    feats, gamma, mask = _tiny_case(4)
    th = _rand_theta(5, scale=1.0)
    loss, grad, _ = cnn.loss_and_grad(th, feats, gamma, mask, rounding=False)
    f = lambda t: cnn.loss_and_grad(t, feats, gamma, mask, rounding=False)[0]  # noqa: E731
    rng = np.random.default_rng(6)
    # a few coordinates of every layer's W and b
    offs, k = [], 0
    for ws, bs in cnn.layer_shapes():
        nw = int(np.prod(ws))
        offs += list(k + rng.choice(nw, 4, replace=False)) + [k + nw + int(rng.integers(bs[0]))]
        k += nw + bs[0]
    h = 1e-6
    for i in offs:
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (f(tp) - f(tm)) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-5 * max(abs(fd), 1e-3), (i, fd, grad[i])


def test_receptive_field_and_patch_equivalence():
    feats, _, _ = _tiny_case(7, shape=(11, 12, 10))
    th = _rand_theta(8)
    y = cnn.forward(th, feats).y
    # the value at a node is the network on its own 9x9x9 patch of the padded input
    fp = cnn.pad(feats)
    for p in [(0, 0, 0), (5, 6, 4), (10, 11, 9), (3, 0, 9)]:
        patch = fp[:, p[0]:p[0] + 9, p[1]:p[1] + 9, p[2]:p[2] + 9]
        # valid convolutions straight over the patch (no further padding)
        x = cnn.bf16(patch)
        for l, (w, b) in enumerate(cnn.unflatten(th)):
            z = cnn.conv3d_valid(x, cnn.bf16(w), b.astype(np.float32).astype(np.float64))
            x = cnn.bf16(np.maximum(z, 0)) if l < 3 else z
        assert x.shape == (1, 1, 1, 1)
        assert x[0, 0, 0, 0] == y[p]
    # perturbing one input node changes exactly the outputs within Chebyshev distance 4
    q = (6, 5, 5)
    f2 = feats.copy()
    f2[1][q] += 3.0
    y2 = cnn.forward(th, f2, rounding=False).y
    y1 = cnn.forward(th, feats, rounding=False).y
    zz, yy, xx = np.meshgrid(*[np.arange(n) for n in y.shape], indexing="ij")
    cheb = np.maximum(np.maximum(abs(zz - q[0]), abs(yy - q[1])), abs(xx - q[2]))
    assert np.all(y2[cheb > 4] == y1[cheb > 4])
    assert np.mean(y2[cheb <= 4] != y1[cheb <= 4]) > 0.5


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, 1.0 + 2.0 ** -7 + 2.0 ** -8,
                     -2.5, 3.0e-40, 65504.0, 1.0 - 2.0 ** -10])
    want = np.array([1.0, 1.0, 1.0 + 2.0 ** -7, 1.0 + 2.0 ** -6, -2.5, None, 65536.0, 1.0], dtype=object)
    got = cnn.bf16(vals)
    for g, w in zip(got, want):
        if w is not None:
            assert g == w
    rng = np.random.default_rng(9)
    x = (rng.normal(size=100000) * np.exp(rng.normal(size=100000) * 5)).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(cnn.bf16(x), ref)


def test_features_in_float32_steps():
    rng = np.random.default_rng(10)
    ref = rng.uniform(0, 2, size=(3, 4, 5)).astype(np.float32)
    ev = (ref + rng.normal(size=ref.shape) * 0.02).astype(np.float32)
    f = cnn.features(ref, ev, 0.03)
    dmax = ref.max()
    assert f[0].max() == 1.0
    # close to the exact quantities, within bf16 rounding
    np.testing.assert_allclose(f[0], ref / dmax, rtol=2 ** -8)
    np.testing.assert_allclose(f[1], (ev.astype(np.float64) - ref) / (0.03 * dmax), rtol=2 ** -8 + 1e-6,
                               atol=1e-6)


def test_adam_closed_forms():
    # constant gradient: bias correction makes m_hat = g and v_hat = g^2 at every step,
    # so each step moves every coordinate by lr * g / (|g| + eps)
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    th = np.array([1.0, 1.0, 1.0, 1.0])
    st = cnn.adam_init(4)
    lr = 0.01
    for t in range(1, 6):
        th = cnn.adam_step(th, g, st, lr)
        np.testing.assert_allclose(th, 1.0 - t * lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # a gradient that flips sign: m_hat after two steps is the bias-corrected mix
    st = cnn.adam_init(1)
    th = cnn.adam_step(np.zeros(1), np.array([1.0]), st, 1.0, beta1=0.5, beta2=0.75, eps=0.0)
    th = cnn.adam_step(th, np.array([-1.0]), st, 1.0, beta1=0.5, beta2=0.75, eps=0.0)
    # step 1: m = 0.5, v = 0.25 -> m_hat = v_hat = 1, theta = -1
    # step 2: m = 0.5*0.5 - 0.5 = -0.25 -> m_hat = -0.25/(1-0.25) = -1/3;
    #         v = 0.75*0.25 + 0.25 = 0.4375 -> v_hat = 0.4375/(1-0.5625) = 1
    np.testing.assert_allclose(th, [-1.0 + 1.0 / 3.0], rtol=1e-14)


@pytest.mark.parametrize("mistake", ["no_relu_mask", "untransposed", "bias_sum"])
def test_planted_backward_mistakes_fail_the_fd_check(mistake, monkeypatch):
    feats, gamma, mask = _tiny_case(11, shape=(5, 6, 5))
    th = _rand_theta(12)
    orig_bwd_data = cnn.conv3d_bwd_data
    orig_bwd_w = cnn.conv3d_bwd_weight
    if mistake == "no_relu_mask":
        monkeypatch.setattr(cnn, "loss_and_grad", _loss_without_relu_mask)
    elif mistake == "untransposed":
        def bd(g, w, in_shape):
            return orig_bwd_data(g, np.flip(w, axis=(2, 3, 4)), in_shape)
        monkeypatch.setattr(cnn, "conv3d_bwd_data", bd)
    else:
        def bw(x, g, ksize=3):
            gw, gb = orig_bwd_w(x, g, ksize)
            return gw, gb * 0.5
        monkeypatch.setattr(cnn, "conv3d_bwd_weight", bw)
    _, grad, _ = cnn.loss_and_grad(th, feats, gamma, mask, rounding=False)
    monkeypatch.undo()
    _, good, _ = cnn.loss_and_grad(th, feats, gamma, mask, rounding=False)
    f = lambda t: cnn.loss_and_grad(t, feats, gamma, mask, rounding=False)[0]  # noqa: E731
    # the finite-difference check over all biases and a sample of weights catches it
    rng = np.random.default_rng(13)
    idx = []
    k = 0
    for ws, bs in cnn.layer_shapes():
        nw = int(np.prod(ws))
        idx += list(k + rng.choice(nw, 6, replace=False)) + list(range(k + nw, k + nw + bs[0]))
        k += nw + bs[0]
    h = 1e-6
    bad_found = False
    for i in idx:
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (f(tp) - f(tm)) / (2 * h)
        assert abs(fd - good[i]) <= 1e-5 * max(abs(fd), 1e-3)
        if abs(fd - grad[i]) > 1e-5 * max(abs(fd), 1e-3):
            bad_found = True
    assert bad_found


def _loss_without_relu_mask(theta, feats, gamma, mask, rounding=True):
    """loss_and_grad with the ReLU backward mask left out (a planted mistake)."""
    fw = cnn.forward(theta, feats, rounding)
    params = cnn.unflatten(theta)
    m = np.asarray(mask, dtype=bool)
    cnt = max(int(m.sum()), 1)
    t = np.where(m, cnn.target(np.where(m, gamma, 1.0)), 0.0)
    r = np.where(m, fw.y - t, 0.0)
    g = (2.0 / cnt) * r[None]
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        w, _ = params[l]
        gw, gb = cnn.conv3d_bwd_weight(fw.inputs[l], g)
        grads[l] = (gw, gb)
        if l > 0:
            g = cnn.conv3d_bwd_data(g, w, fw.inputs[l].shape[1:])
    return float((r * r).sum() / cnt), cnn.flatten(grads), fw


# ---- pooled input (a grid at half the training spacing) ---------------------------------

def test_pool2_brute_force_odd_and_even_shapes():
    rng = np.random.default_rng(70)
    for shape in ((3, 5, 4), (4, 2, 6), (1, 3, 2)):
        v = rng.uniform(0.0, 2.0, size=shape)
        got = cnn.pool2(v)
        want = np.zeros(tuple((n + 1) // 2 for n in shape))
        for cz in range(want.shape[0]):
            for cy in range(want.shape[1]):
                for cx in range(want.shape[2]):
                    vals = [v[z, y, x] for z in (2 * cz, 2 * cz + 1) for y in (2 * cy, 2 * cy + 1)
                            for x in (2 * cx, 2 * cx + 1)
                            if z < shape[0] and y < shape[1] and x < shape[2]]
                    want[cz, cy, cx] = sum(vals) / len(vals)
        assert np.allclose(got, want, rtol=0, atol=1e-15)


def test_pool2_preserves_constants_and_even_sums():
    assert np.all(cnn.pool2(np.full((5, 7, 3), 1.25)) == 1.25)
    v = np.random.default_rng(71).uniform(size=(6, 4, 8))
    assert np.isclose(8.0 * cnn.pool2(v).sum(), v.sum(), rtol=1e-14)


def test_upsample_reproduces_linear_gamma_and_clamps_at_edges():
    """exp(y) interpolated trilinearly: a positive linear function of the coarse index is
    reproduced exactly at every fine node, with the coarse position (p - 1/2) / 2 clamped
    to the coarse grid."""
    fine = (9, 8, 11)
    cz, cy, cx = [(n + 1) // 2 for n in fine]
    a, b = 2.0, np.array([0.3, -0.1, 0.05])
    kz, ky, kx = np.meshgrid(np.arange(cz), np.arange(cy), np.arange(cx), indexing="ij")
    yc = np.log(a + b[0] * kz + b[1] * ky + b[2] * kx)
    nodes = np.arange(np.prod(fine))
    got = np.exp(cnn.upsample_at(yc, fine, nodes))
    z, y, x = np.unravel_index(nodes, fine)
    u = [np.clip((p - 0.5) / 2.0, 0, c - 1) for p, c in ((z, cz), (y, cy), (x, cx))]
    want = a + b[0] * u[0] + b[1] * u[1] + b[2] * u[2]
    assert np.allclose(got, want, rtol=1e-13, atol=0)
    # node 0 clamps to coarse node 0 on every axis; constants stay constant
    assert np.isclose(got[0], np.exp(yc[0, 0, 0]), rtol=1e-14)
    assert np.allclose(cnn.upsample_at(np.full((cz, cy, cx), -0.7), fine, nodes), -0.7, rtol=0, atol=1e-15)


def test_pooled_forward_of_block_constant_pair_is_the_coarse_network():
    """A fine pair that is constant on every 2x2x2 block pools back to the coarse pair, so
    the pooled network is the network on the coarse pair (same Dmax)."""
    rng = np.random.default_rng(72)
    cref = rng.uniform(0.1, 2.0, size=(6, 5, 7)).astype(np.float32)
    cev = (cref * rng.uniform(0.9, 1.1, size=cref.shape)).astype(np.float32)
    rep = lambda c: np.repeat(np.repeat(np.repeat(c, 2, 0), 2, 1), 2, 2)
    th = cnn.init_params(73)
    got = cnn.pooled_forward(th, rep(cref), rep(cev), 0.03).y
    want = cnn.forward(th, cnn.features(cref, cev, 0.03)).y
    assert np.array_equal(got, want)
