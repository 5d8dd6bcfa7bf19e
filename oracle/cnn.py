"""FP64 CPU oracle of the learned search radius (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use this
module; the GPU library neither imports nor links it.

The network (not described in the paper; an addition around its method): a small 3D CNN
maps each node's 9x9x9 neighbourhood of two dose features to a prediction of
log(gamma + 0.01) at that node.

* Input features at every grid node, in float32 steps:
    f0 = fl32(D_r * fl32(1 / Dmax))                      (reference dose, normalised)
    f1 = fl32(fl32(D_e - D_r) * fl32(1 / fl32(DD * Dmax))) (signed gamma0, global dD)
  each rounded to bfloat16; outside the grid both are 0 (zero padding by 4 nodes).
* Four valid 3x3x3 convolutions, channels 2 -> 16 -> 16 -> 16 -> 1, ReLU after the
  first three, none after the last:  out[o, p] = b[o] + sum_{i, t} w[o, i, t] x[i, p + t].
  With the input padded by 4 the output covers the grid; its value at a node depends
  on exactly that node's 9x9x9 input patch.
* Arithmetic points (the GPU kernels take the same ones): products use the bfloat16
  values (round to nearest even) of the FP32 master weights; every hidden activation is
  rounded to bfloat16 after its ReLU; biases and the last layer's output stay FP32.
  This oracle sums in FP64 (the kernels in FP32), so a sum that lands next to a
  bfloat16 rounding boundary may round the other way: the tests bound that.
* Training: loss = mean over masked nodes of (y - log(gamma + 0.01))^2; gradients by
  the chain rule written out (bwd-data = full correlation with the flipped, transposed
  kernel; bwd-weight = correlation of the layer input with the output gradient; ReLU
  passes the gradient where its stored output is > 0); Adam (Kingma & Ba 2015) with bias
  correction on the FP32 master weights.  The output gradient of every layer is rounded
  to bfloat16 (it is a matrix-core operand in the kernels); the weight gradients are
  exact sums of those bf16 products here, FP32 sums in the kernels.

* Pooled input (for a grid at half the spacing the network was trained on): the pair is
  averaged over 2x2x2 blocks onto the coarse grid ceil(n / 2) per axis (a block at an odd
  edge averages the fine nodes it holds), the features use the fine grid's Dmax, the
  network runs on the coarse grid, and at a fine node p the coarse values of
  gamma_hat + 0.01 = exp(y) are interpolated trilinearly at coarse position (p - 1/2) / 2
  per axis (coarse node k sits at fine position 2k + 1/2), clamped to the coarse grid.

Parameter layout (one flat float array, the order the C ABI uses): for each layer l,
W_l[co][ci][dz][dy][dx] followed by b_l[co].
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np

CHANNELS = (2, 16, 16, 16, 1)
KSIZE = 3
PAD = 4                      # = number of layers * (KSIZE // 2)
GAMMA_EPS = 0.01             # target = log(gamma + GAMMA_EPS)


def layer_shapes() -> List[Tuple[Tuple[int, ...], Tuple[int]]]:
    return [((co, ci, KSIZE, KSIZE, KSIZE), (co,)) for ci, co in zip(CHANNELS[:-1], CHANNELS[1:])]


def n_params() -> int:
    return sum(int(np.prod(w)) + b[0] for w, b in layer_shapes())


def unflatten(theta: np.ndarray) -> List[Tuple[np.ndarray, np.ndarray]]:
    """Flat parameter vector -> [(W_l, b_l)] (views in FP64)."""
    theta = np.asarray(theta, dtype=np.float64)
    out, k = [], 0
    for ws, bs in layer_shapes():
        nw = int(np.prod(ws))
        out.append((theta[k:k + nw].reshape(ws), theta[k + nw:k + nw + bs[0]]))
        k += nw + bs[0]
    assert k == theta.size
    return out


def flatten(params: Sequence[Tuple[np.ndarray, np.ndarray]]) -> np.ndarray:
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params])


def bf16(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), via float32; returned as float64."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def features(ref: np.ndarray, ev: np.ndarray, dd: float, dose_max: float = None) -> np.ndarray:
    """The two input channels on the grid (before padding), float32 steps then bf16."""
    ref = np.asarray(ref, dtype=np.float32)
    ev = np.asarray(ev, dtype=np.float32)
    dmax = np.float32(ref.max() if dose_max is None else dose_max)
    inv_max = np.float32(1.0) / dmax
    inv_dd = np.float32(1.0) / np.float32(np.float32(dd) * dmax)
    f0 = ref * inv_max
    f1 = (ev - ref) * inv_dd
    return np.stack([bf16(f0), bf16(f1)])


def pad(x: np.ndarray, p: int = PAD) -> np.ndarray:
    return np.pad(x, [(0, 0)] + [(p, p)] * (x.ndim - 1))


def conv3d_valid(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """out[o, z, y, x] = b[o] + sum_{i,dz,dy,dx} w[o,i,dz,dy,dx] x[i, z+dz, y+dy, x+dx]."""
    ci, Z, Y, X = x.shape
    co, ci2, kz, ky, kx = w.shape
    assert ci == ci2
    oz, oy, ox = Z - kz + 1, Y - ky + 1, X - kx + 1
    out = np.broadcast_to(b.reshape(co, 1, 1, 1), (co, oz, oy, ox)).astype(np.float64)
    for dz in range(kz):
        for dy in range(ky):
            for dx in range(kx):
                patch = x[:, dz:dz + oz, dy:dy + oy, dx:dx + ox].reshape(ci, -1)
                out = out + (w[:, :, dz, dy, dx] @ patch).reshape(co, oz, oy, ox)
    return out


def conv3d_bwd_data(g: np.ndarray, w: np.ndarray, in_shape) -> np.ndarray:
    """d loss / d x for out = conv3d_valid(x, w, b), given g = d loss / d out."""
    co, oz, oy, ox = g.shape
    _, ci, kz, ky, kx = w.shape
    gx = np.zeros((ci,) + tuple(in_shape), dtype=np.float64)
    gf = g.reshape(co, -1)
    for dz in range(kz):
        for dy in range(ky):
            for dx in range(kx):
                gx[:, dz:dz + oz, dy:dy + oy, dx:dx + ox] += (w[:, :, dz, dy, dx].T @ gf).reshape(ci, oz, oy, ox)
    return gx


def conv3d_bwd_weight(x: np.ndarray, g: np.ndarray, ksize: int = KSIZE):
    """(d loss / d w, d loss / d b) for out = conv3d_valid(x, w, b)."""
    ci = x.shape[0]
    co, oz, oy, ox = g.shape
    gw = np.zeros((co, ci, ksize, ksize, ksize), dtype=np.float64)
    gf = g.reshape(co, -1)
    for dz in range(ksize):
        for dy in range(ksize):
            for dx in range(ksize):
                patch = x[:, dz:dz + oz, dy:dy + oy, dx:dx + ox].reshape(ci, -1)
                gw[:, :, dz, dy, dx] = gf @ patch.T
    return gw, gf.sum(axis=1)


@dataclass
class Forward:
    inputs: List[np.ndarray]     # the input of each layer (bf16 values; the first is padded)
    pre: List[np.ndarray]        # each layer's output before ReLU / rounding
    y: np.ndarray                # last layer output (grid shape)


def forward(theta: np.ndarray, feats: np.ndarray, rounding: bool = True, padded: bool = False) -> Forward:
    """Run the network on features of shape (2, Z, Y, X); returns every activation.

    padded=False pads the features with zeros by 4 nodes (output shape = input shape);
    padded=True takes them as given (a crop with its neighbourhood: output 8 smaller).
    rounding=False drops the bf16 rounding of weights and activations and the FP32
    rounding of the biases (exact FP64 network) - used by the finite-difference checks.
    """
    rnd = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    f32 = (lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)) if rounding else rnd
    params = unflatten(theta)
    x = rnd(feats) if padded else pad(rnd(feats))
    inputs, pre = [], []
    for l, (w, b) in enumerate(params):
        inputs.append(x)
        z = conv3d_valid(x, rnd(w), f32(b))
        pre.append(z)
        if l + 1 < len(params):
            x = rnd(np.maximum(z, 0.0))
    return Forward(inputs, pre, pre[-1][0])


def target(gamma: np.ndarray) -> np.ndarray:
    return np.log(np.asarray(gamma, dtype=np.float64) + GAMMA_EPS)


def loss_and_grad(theta: np.ndarray, feats: np.ndarray, gamma: np.ndarray, mask: np.ndarray,
                  rounding: bool = True, padded: bool = False, count: int = None):
    """Masked mean-squared error on log(gamma + 0.01) and its gradient (flat, FP64).

    count: the number of nodes the mean runs over (default: the masked nodes here; a
    batch of crops shares the count of the whole batch).
    """
    rnd = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    fw = forward(theta, feats, rounding, padded)
    params = unflatten(theta)
    m = np.asarray(mask, dtype=bool)
    cnt = max(int(m.sum()), 1) if count is None else count
    t = np.where(m, target(np.where(m, gamma, 1.0)), 0.0)
    r = np.where(m, fw.y - t, 0.0)
    loss = float((r * r).sum() / cnt)
    g = rnd((2.0 / cnt) * r[None])                  # d loss / d (last layer output)
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        w, _ = params[l]
        x = fw.inputs[l]
        gw, gb = conv3d_bwd_weight(x, g)
        grads[l] = (gw, gb)
        if l > 0:
            gx = conv3d_bwd_data(g, rnd(w), x.shape[1:])
            # ReLU of the previous layer: the gradient passes where the stored activation
            # (this layer's input) is positive
            g = rnd(gx * (x > 0.0))
    return loss, flatten(grads), fw


@dataclass
class AdamState:
    m: np.ndarray
    v: np.ndarray
    t: int = 0


def adam_init(n: int) -> AdamState:
    return AdamState(np.zeros(n), np.zeros(n), 0)


def adam_step(theta: np.ndarray, grad: np.ndarray, st: AdamState, lr: float,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> np.ndarray:
    """One Adam update (Kingma & Ba 2015, Algorithm 1) in FP64; returns the new theta."""
    st.t += 1
    st.m = beta1 * st.m + (1.0 - beta1) * grad
    st.v = beta2 * st.v + (1.0 - beta2) * grad * grad
    mhat = st.m / (1.0 - beta1 ** st.t)
    vhat = st.v / (1.0 - beta2 ** st.t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps)


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases (FP32 values), as a flat FP64 vector."""
    rng = np.random.default_rng(seed)
    parts = []
    for ws, bs in layer_shapes():
        fan_in = ws[1] * ws[2] * ws[3] * ws[4]
        lim = np.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, size=ws).astype(np.float32).ravel())
        parts.append(np.zeros(bs, dtype=np.float32))
    return np.concatenate(parts).astype(np.float64)


def predict_gamma(theta: np.ndarray, ref: np.ndarray, ev: np.ndarray, dd: float) -> np.ndarray:
    """gamma_hat = max(exp(y) - 0.01, 0) at every grid node."""
    y = forward(theta, features(ref, ev, dd)).y
    return np.maximum(np.exp(y) - GAMMA_EPS, 0.0)


def pool2(vol: np.ndarray) -> np.ndarray:
    """FP64 mean over each 2x2x2 block of a 3D volume (ceil(n / 2) blocks per axis; a block
    at an odd edge averages the nodes it holds)."""
    v = np.asarray(vol, dtype=np.float64)
    cz, cy, cx = [(n + 1) // 2 for n in v.shape]
    total = np.zeros((cz, cy, cx))
    count = np.zeros((cz, cy, cx))
    for dz in range(2):
        for dy in range(2):
            for dx in range(2):
                part = v[dz::2, dy::2, dx::2]
                total[:part.shape[0], :part.shape[1], :part.shape[2]] += part
                count[:part.shape[0], :part.shape[1], :part.shape[2]] += 1.0
    return total / count


def pooled_axis(p: np.ndarray, c: int):
    """Trilinear interpolation on one axis: lower coarse index, upper index and weight of
    the upper one for fine indices p (coarse node k at fine position 2k + 1/2)."""
    u = np.clip((np.asarray(p, dtype=np.float64) - 0.5) / 2.0, 0.0, c - 1.0)
    i0 = np.minimum(np.floor(u).astype(np.int64), c - 1)
    i1 = np.minimum(i0 + 1, c - 1)
    return i0, i1, u - i0


def upsample_at(yc: np.ndarray, fine_shape, nodes: np.ndarray) -> np.ndarray:
    """y at flat fine-grid node indices from the coarse output yc: exp(yc) interpolated
    trilinearly, then log."""
    nz, ny, nx = fine_shape
    nodes = np.asarray(nodes, dtype=np.int64)
    z, y, x = nodes // (ny * nx), (nodes // nx) % ny, nodes % nx
    cz, cy, cx = yc.shape
    z0, z1, tz = pooled_axis(z, cz)
    y0, y1, ty = pooled_axis(y, cy)
    x0, x1, tx = pooled_axis(x, cx)
    g = np.exp(np.asarray(yc, dtype=np.float64))
    val = np.zeros(len(nodes))
    for zi, wz in ((z0, 1.0 - tz), (z1, tz)):
        for yi, wy in ((y0, 1.0 - ty), (y1, ty)):
            for xi, wx in ((x0, 1.0 - tx), (x1, tx)):
                val += wz * wy * wx * g[zi, yi, xi]
    return np.log(val)


def pooled_forward(theta: np.ndarray, ref: np.ndarray, ev: np.ndarray, dd: float) -> Forward:
    """The network on the pooled pair's coarse grid (features with the fine Dmax)."""
    dmax = float(np.asarray(ref, dtype=np.float32).max())
    f = features(pool2(ref).astype(np.float32), pool2(ev).astype(np.float32), dd, dose_max=dmax)
    return forward(theta, f)


def predict_pooled_at(theta: np.ndarray, ref: np.ndarray, ev: np.ndarray, dd: float,
                      nodes: np.ndarray) -> np.ndarray:
    """y = log(gamma_hat + 0.01) at fine nodes from the pooled input."""
    return upsample_at(pooled_forward(theta, ref, ev, dd).y, np.shape(ref), nodes)
