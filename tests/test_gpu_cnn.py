"""GPU parity of the learned-radius CNN kernels (through the C ABI) against the FP64 oracle.

Tolerances.  The kernels and the oracle take the same bf16 rounding points; they differ
in the summation (FP32 in the kernels, exact here).  A sum that lands next to a bf16
rounding boundary may round the other way, so a hidden activation can differ by one bf16
ulp (2^-8 relative).  Propagated through the remaining layers that bounds the output
difference at a node by (number of rounded layers) * 2^-8 * A, where A is the same network
evaluated on absolute values (|b| + sum |w| |x|): the largest any partial sum can be.  The
tests use 4 * 2^-8 * A.  Gradients: each product has bf16 operands on both sides, so the
error comes from FP32 summation and the same rare one-ulp flips; the tests bound the
relative L2 error per layer by 2^-6 (a dropped tap or channel of one layer moves it by
more than 1/27) and every element by 5 % of the layer's largest gradient.
"""
import os

import numpy as np
import pytest

from gpu_util import dev, host
from oracle import cnn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gx():
    import paper_1012_1900_amd as g
    return g


def _theta(seed):
    th = cnn.init_params(seed)
    rng = np.random.default_rng(seed + 1)
    k = 0
    for ws, bs in cnn.layer_shapes():
        k += int(np.prod(ws))
        th[k:k + bs[0]] = rng.uniform(-0.2, 0.2, bs[0]).astype(np.float32)
        k += bs[0]
    return th


def _bf16_bits(x):
    """Random inputs as bf16 values: truncate float32 to its top 16 bits."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32)
    return (u >> 16).astype(np.uint16)


def _bits_to_f64(b):
    return (b.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _feat_tensor(bits):
    import torch
    return torch.from_numpy(np.ascontiguousarray(bits).view(np.int16)).to("cuda")


def _abs_network(theta, feats, padded=False):
    """|b| + sum |w| |x| layer by layer (no rounding): bounds every partial sum."""
    x = np.abs(feats) if padded else cnn.pad(np.abs(feats))
    for l, (w, b) in enumerate(cnn.unflatten(theta)):
        x = cnn.conv3d_valid(x, np.abs(w), np.abs(b))
    return x[0]


def _random_crops(seed, nvol, crop):
    rng = np.random.default_rng(seed)
    shape = (nvol,) + tuple(c + 8 for c in crop) + (2,)
    f = rng.normal(size=shape).astype(np.float32)
    f[..., 0] = np.abs(f[..., 0])
    return _bf16_bits(f)


@pytest.mark.parametrize("crop", [(13, 17, 21), (4, 9, 33), (1, 1, 1)])
def test_forward_parity(gx, crop):
    th = _theta(1)
    bits = _random_crops(2, 3, crop)
    m = gx.Model(th.astype(np.float32))
    y = host(m.forward(_feat_tensor(bits)))
    for v in range(bits.shape[0]):
        f = np.moveaxis(_bits_to_f64(bits[v]), -1, 0)
        want = cnn.forward(th, f, padded=True).y
        bound = 4 * 2.0 ** -8 * _abs_network(th, f, padded=True) + 1e-6
        err = np.abs(y[v] - want)
        assert np.all(err <= bound), (v, float(err.max()), float((err / bound).max()))
        # most nodes agree to FP32 summation accuracy
        assert np.mean(err <= 1e-4 * bound / (4 * 2.0 ** -8)) > 0.95
        # ... measured against the output itself: the bound above grows with the network's
        # absolute values and would let a dropped tap through; one-ulp bf16 flips of hidden
        # activations stay rare, so 95 % of the nodes match to 1e-3 of the output's range
        assert np.quantile(err, 0.95) <= 1e-3 * (1.0 + np.abs(want).max()), (v, float(np.quantile(err, 0.95)))


def _pair(seed, shape=(22, 25, 29)):
    from dosegen import make_pair_3d
    return make_pair_3d(seed, shape=shape, spacing=(2.5, 2.5, 2.5))


def test_features_bit_exact(gx):
    pair = _pair(3)
    ref, ev = dev(pair.ref), dev(pair.eval)
    feat = host(gx.model_features(ref, ev, pair.spacing, 0.03)).view(np.uint16)
    want = cnn.pad(cnn.features(pair.ref, pair.eval, 0.03))
    want_bits = (want.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    assert np.array_equal(feat, np.moveaxis(want_bits, 0, -1))


def test_predict_full_grid(gx):
    pair = _pair(4)
    th = _theta(5)
    m = gx.Model(th.astype(np.float32))
    y = host(m.predict(dev(pair.ref), dev(pair.eval), pair.spacing, 0.03))
    f = cnn.features(pair.ref, pair.eval, 0.03)
    want = cnn.forward(th, f).y
    bound = 4 * 2.0 ** -8 * _abs_network(th, f) + 1e-6
    assert np.all(np.abs(y - want) <= bound)
    assert np.quantile(np.abs(y - want), 0.95) <= 1e-3 * (1.0 + np.abs(want).max())


def _labels(seed, nvol, crop):
    rng = np.random.default_rng(seed)
    g = np.exp(rng.normal(size=(nvol,) + crop) * 0.7) * 0.4
    mask = rng.uniform(size=g.shape) < 0.6
    return np.where(mask, g, -1.0).astype(np.float32)


def _oracle_batch_grad(th, bits, labels):
    # the loss is a mean over every labelled node of the batch
    cnt_all = int((labels >= 0).sum())
    tot_loss, grads = 0.0, np.zeros_like(th)
    for v in range(bits.shape[0]):
        f = np.moveaxis(_bits_to_f64(bits[v]), -1, 0)
        m = labels[v] >= 0
        loss, grad, _ = cnn.loss_and_grad(th, f, labels[v].astype(np.float64), m, padded=True, count=cnt_all)
        tot_loss += loss
        grads += grad
    return tot_loss, grads


def test_train_step_gradient_parity(gx):
    crop = (6, 10, 19)
    th = _theta(7)
    bits = _random_crops(8, 2, crop)
    labels = _labels(9, 2, crop)
    m = gx.Model(th.astype(np.float32))
    loss = m.train_step(_feat_tensor(bits), dev(labels), lr=0.0)
    g_gpu = m.grad().astype(np.float64)
    want_loss, g_ref = _oracle_batch_grad(th, bits, labels)
    assert abs(loss - want_loss) <= 1e-3 * want_loss
    off = 0
    for l, (ws, bs) in enumerate(cnn.layer_shapes()):
        n = int(np.prod(ws)) + bs[0]
        a, b = g_gpu[off:off + n], g_ref[off:off + n]
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        assert rel <= 2.0 ** -6, (l, rel)
        assert np.max(np.abs(a - b)) <= 0.05 * np.max(np.abs(b)), l
        off += n
    # lr = 0 leaves the parameters as they were
    assert np.array_equal(m.params(), th.astype(np.float32))


def test_adam_step_parity(gx):
    crop = (5, 8, 16)
    th = _theta(10)
    bits = _random_crops(11, 2, crop)
    labels = _labels(12, 2, crop)
    lr = 1e-3
    m = gx.Model(th.astype(np.float32))
    m.train_step(_feat_tensor(bits), dev(labels), lr=lr)
    p_gpu = m.params().astype(np.float64)
    _, g_ref = _oracle_batch_grad(th, bits, labels)
    st = cnn.adam_init(th.size)
    want = cnn.adam_step(th.astype(np.float32).astype(np.float64), g_ref, st, lr)
    d = np.abs(p_gpu - want)
    # first step: each parameter moves by lr * g / (|g| + eps), i.e. by ~lr where the
    # gradient is clearly non-zero; only its sign matters there
    big = np.abs(g_ref) > 0.05 * np.max(np.abs(g_ref))
    assert np.all(d[big] <= 1e-3 * lr + 1e-7)
    assert np.all(d <= 2 * lr + 1e-7)


def test_training_lowers_the_loss(gx):
    crop = (8, 8, 16)
    th = _theta(13)
    bits = _random_crops(14, 4, crop)
    labels = _labels(15, 4, crop)
    m = gx.Model(th.astype(np.float32))
    f, lab = _feat_tensor(bits), dev(labels)
    losses = [m.train_step(f, lab, lr=3e-3) for _ in range(40)]
    assert losses[-1] < 0.5 * losses[0], losses[::8]


def test_predict_at_listed_nodes(gx):
    """The network at listed nodes only (each from its own 9^3 patch), as the learned
    search evaluates it: the oracle's whole-grid values at those nodes, and the GPU's own
    whole-grid pass there up to the order of the last layer's sum."""
    import torch
    pair = _pair(6)
    th = _theta(9)
    m = gx.Model(th.astype(np.float32))
    ref, ev = dev(pair.ref), dev(pair.eval)
    n = pair.ref.size
    rng = np.random.default_rng(10)
    nz, ny, nx = pair.ref.shape
    corners = [((z * ny) + y) * nx + x for z in (0, nz - 1) for y in (0, ny - 1) for x in (0, nx - 1)]
    nodes = np.unique(np.concatenate([rng.choice(n, 400, replace=False), corners])).astype(np.int32)
    y = host(gx.predict_nodes(m, ref, ev, pair.spacing, 0.03, torch.from_numpy(nodes).to("cuda")))
    f = cnn.features(pair.ref, pair.eval, 0.03)
    want = cnn.forward(th, f).y.ravel()[nodes]
    A = _abs_network(th, f).ravel()[nodes]
    assert np.all(np.abs(y - want) <= 4 * 2.0 ** -8 * A + 1e-6)
    dense = host(m.predict(ref, ev, pair.spacing, 0.03)).ravel()[nodes]
    assert np.all(np.abs(y - dense) <= 1e-5 * A + 1e-6)


def test_predict_pooled_at_listed_nodes(gx):
    """The pooled input (gammax_model_predict_nodes_pooled): the pair averaged 2x2x2, the
    network on the coarse grid, exp(y) interpolated trilinearly at the fine nodes.  Against
    the oracle, within the bf16 bound of the 8 coarse corners of each node (the log of an
    interpolated exp moves by at most the largest corner error); odd and even axes."""
    import torch
    from dosegen import make_pair_3d
    pair = make_pair_3d(8, shape=(25, 30, 27), spacing=(1.25, 1.25, 1.25))
    th = _theta(11)
    m = gx.Model(th.astype(np.float32))
    ref, ev = dev(pair.ref), dev(pair.eval)
    n = pair.ref.size
    rng = np.random.default_rng(12)
    nz, ny, nx = pair.ref.shape
    corners = [((z * ny) + y) * nx + x for z in (0, nz - 1) for y in (0, ny - 1) for x in (0, nx - 1)]
    nodes = np.unique(np.concatenate([rng.choice(n, 600, replace=False), corners])).astype(np.int32)
    y = host(gx.predict_nodes(m, ref, ev, pair.spacing, 0.03, torch.from_numpy(nodes).to("cuda"), pool=2))
    want = cnn.predict_pooled_at(th, pair.ref, pair.eval, 0.03, nodes)
    dmax = float(pair.ref.max())
    fc = cnn.features(cnn.pool2(pair.ref).astype(np.float32), cnn.pool2(pair.eval).astype(np.float32), 0.03,
                      dose_max=dmax)
    A = _abs_network(th, fc)
    z, yy, x = np.unravel_index(nodes.astype(np.int64), pair.ref.shape)
    bound = np.zeros(len(nodes))
    axes = [cnn.pooled_axis(p, c) for p, c in ((z, A.shape[0]), (yy, A.shape[1]), (x, A.shape[2]))]
    for zi in axes[0][:2]:
        for yi in axes[1][:2]:
            for xi in axes[2][:2]:
                bound = np.maximum(bound, A[zi, yi, xi])
    assert np.all(np.abs(y - want) <= 4 * 2.0 ** -8 * bound + 1e-5)


def test_model_save_load(gx, tmp_path):
    """Parameters round-trip through a .npy file bit for bit."""
    m = gx.Model(_theta(11))
    path = str(tmp_path / "theta.npy")
    m.save_params(path)
    m2 = gx.Model.load(path)
    assert np.array_equal(m.params(), m2.params())
    assert np.array_equal(m2.params(), np.asarray(_theta(11), dtype=np.float32).ravel())


def test_checkpoint_resumes_training(gx, tmp_path):
    """gammax_model_save / _load keep the parameters and the Adam state: a model loaded after
    three steps takes the next two steps exactly as the original does (same losses, same
    parameters), while a model given only the parameters (fresh Adam state) does not."""
    crop = (8, 8, 16)
    m = gx.Model(_theta(21).astype(np.float32))
    batches = [(_feat_tensor(_random_crops(30 + k, 3, crop)), dev(_labels(40 + k, 3, crop))) for k in range(5)]
    for f, lab in batches[:3]:
        m.train_step(f, lab, lr=2e-3)
    path = str(tmp_path / "model.ckpt")
    m.save(path)
    head = open(path, "rb").readline().decode()
    assert '"format": "gammax-model"' in head and '"adam_step": 3' in head
    assert os.path.getsize(path) == len(head.encode()) + 3 * 4 * gx.MODEL_NPARAM
    m2 = gx.Model.load(path)
    assert np.array_equal(m.params(), m2.params())
    fresh = gx.Model(m.params())
    for f, lab in batches[3:]:
        a, b, c = m.train_step(f, lab, lr=2e-3), m2.train_step(f, lab, lr=2e-3), fresh.train_step(f, lab, lr=2e-3)
        assert a == b
    assert np.array_equal(m.params(), m2.params())
    assert not np.array_equal(m.params(), fresh.params())


def test_checkpoint_rejects_other_files(gx, tmp_path):
    bad = tmp_path / "bad.ckpt"
    bad.write_bytes(b'{"format": "gammax-model", "version": 1, "nparam": 7, "adam_step": 0}\n' + b"\0" * 84)
    with pytest.raises(gx.GammaxError) as e:
        gx.Model.load(str(bad))
    assert e.value.status == -9
    m = gx.Model(_theta(3))
    good = str(tmp_path / "m.ckpt")
    m.save(good)
    raw = open(good, "rb").read()
    (tmp_path / "short.ckpt").write_bytes(raw[:-4])
    with pytest.raises(gx.GammaxError):
        gx.Model.load(str(tmp_path / "short.ckpt"))
    with pytest.raises(gx.GammaxError):
        m.save(str(tmp_path / "no_such_dir" / "m.ckpt"))
