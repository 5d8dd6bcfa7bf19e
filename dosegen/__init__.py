"""Seeded synthetic dose pairs shaped like the IMRT pairs of Gu, Jia & Jiang (Sec. 3.1).

The paper evaluates on eight private IMRT pairs (Monte Carlo reference, pencil-beam
evaluation, normalised to the prescription dose, Sec. 3.1).  They are not available,
so these generators stand in for them.  This module only makes inputs: it holds none
of the gamma-index arithmetic and is shared by the FP64 oracle tests and the GPU path
alike.

Conventions (used by every consumer):
  * arrays are C-ordered float32, shape (ny, nx) in 2D or (nz, ny, nx) in 3D, x fastest;
  * ``spacing`` is given in the same axis order, in millimetres;
  * node i of an axis sits at (i - (n-1)/2) * h, so the box spans n*h millimetres.

Draw order inside each generator is fixed (documented inline) so that a seed maps to
one pair on any machine with the same numpy.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Sequence, Tuple

import numpy as np
from scipy import ndimage

__all__ = [
    "DosePair",
    "make_pair_2d",
    "make_pair_3d",
    "make_config_pair",
    "batch_specs",
    "make_batch_pair",
    "CONFIG_SHAPES",
]

_LN4 = math.log(4.0)


@dataclass
class DosePair:
    ref: np.ndarray          # float32, C-ordered
    eval: np.ndarray         # float32, same shape
    spacing: Tuple[float, ...]
    meta: dict


def _logistic(x: np.ndarray) -> np.ndarray:
    # numerically safe logistic
    return 0.5 * (1.0 + np.tanh(0.5 * x))


def _edge_width(penumbra_mm: float) -> float:
    """Logistic width whose 20 %-80 % rise equals the penumbra."""
    return penumbra_mm / (2.0 * _LN4)


def _soft_interval(coord: np.ndarray, lo: float, hi: float, w: float) -> np.ndarray:
    return _logistic((coord - lo) / w) * _logistic((hi - coord) / w)


def _centred_axes(shape: Sequence[int], spacing: Sequence[float]):
    return [(np.arange(n, dtype=np.float64) - (n - 1) / 2.0) * h for n, h in zip(shape, spacing)]


def _perturb(ref: np.ndarray, spacing, rng: np.random.Generator, hot_spot: bool,
             axes=None) -> Tuple[np.ndarray, dict]:
    """Evaluation dose = shifted, scaled, (hot/cold spotted), noisy copy of ``ref``.

    Draw order: per-axis shift (mm), global scale, [spot centre index, spot sign], noise.
    The shift uses linear interpolation with edge clamping.
    """
    nd = ref.ndim
    shift_mm = rng.uniform(-1.5, 1.5, size=nd)
    scale = rng.uniform(0.97, 1.03)
    ev = ndimage.shift(ref, shift_mm / np.asarray(spacing, dtype=np.float64),
                       order=1, mode="nearest", prefilter=False)
    ev = ev * scale
    meta = {"shift_mm": shift_mm.tolist(), "scale": float(scale)}
    if hot_spot:
        cand = np.flatnonzero(ref.ravel() > 0.5)
        c_lin = int(cand[rng.integers(0, cand.size)])
        sign = 1.0 if rng.integers(0, 2) == 1 else -1.0
        c_idx = np.unravel_index(c_lin, ref.shape)
        r2 = np.zeros(ref.shape, dtype=np.float64)
        for ax in range(nd):
            d = axes[ax] - axes[ax][c_idx[ax]]
            sh = [1] * nd
            sh[ax] = -1
            r2 = r2 + (d * d).reshape(sh)
        ev = ev * (1.0 + sign * 0.05 * np.exp(-r2 / 200.0))   # sigma = 10 mm
        meta.update(spot_index=[int(i) for i in c_idx], spot_sign=sign)
    ev = ev + rng.normal(0.0, 0.005, size=ref.shape)
    return ev, meta


def make_pair_2d(seed: int, shape=(64, 64), spacing=(1.0, 1.0), n_blobs: int = 5) -> DosePair:
    """2D pair: Gaussian blobs inside a sigmoid-edged rectangular field (3 mm penumbra).

    Draw order: rectangle sides (2), rectangle centre (2), then per blob amplitude,
    sigma_y, sigma_x, centre_y, centre_x; then the evaluation perturbation.
    """
    rng = np.random.default_rng(seed)
    yy, xx = _centred_axes(shape, spacing)
    ext = np.array([shape[0] * spacing[0], shape[1] * spacing[1]])
    sides = rng.uniform(0.4, 0.8, size=2) * ext
    centre = rng.uniform(-0.1, 0.1, size=2) * ext
    w = _edge_width(3.0)
    lo = centre - sides / 2
    hi = centre + sides / 2
    field = (_soft_interval(yy, lo[0], hi[0], w)[:, None]
             * _soft_interval(xx, lo[1], hi[1], w)[None, :])
    acc = np.zeros(shape, dtype=np.float64)
    for _ in range(n_blobs):
        amp = rng.uniform(0.3, 1.0)
        sy, sx = rng.uniform(4.0, 15.0, size=2)
        cy = rng.uniform(lo[0], hi[0])
        cx = rng.uniform(lo[1], hi[1])
        acc += amp * np.exp(-((yy - cy) ** 2) / (2 * sy * sy))[:, None] \
            * np.exp(-((xx - cx) ** 2) / (2 * sx * sx))[None, :]
    ref = field * acc
    ref /= ref.max()
    ev, meta = _perturb(ref, spacing, rng, hot_spot=False)
    return DosePair(ref.astype(np.float32), ev.astype(np.float32), tuple(float(s) for s in spacing),
                    dict(meta, generator="2d-blobs", seed=seed))


def make_pair_3d(seed: int, shape=(96, 128, 128), spacing=(2.5, 2.5, 2.5), n_beams: int = 7,
                 hot_spot: bool = True) -> DosePair:
    """3D pair: coplanar beams with segmented sigmoid-edged apertures and exponential
    depth attenuation (0.045 /cm), normalised to max 1.

    Beams rotate about the z axis (slowest array axis); gantry angle of beam k is
    360*k/n + U[0, 51] degrees; rays are parallel and pass the box centre.  Depth is the
    projection on the beam axis plus the in-plane half diagonal of the box.  Each beam's
    aperture is the union (max) of 3-8 rectangles in beam's-eye-view (lateral, z)
    coordinates, sides U[10, 60] mm, centres within +-40 mm, 4 mm penumbra; beam weights
    U[0.5, 1].

    Draw order: per beam: angle jitter, weight, rectangle count, then per rectangle
    lateral side, z side, lateral centre, z centre; then the evaluation perturbation.
    """
    rng = np.random.default_rng(seed)
    zz, yy, xx = _centred_axes(shape, spacing)
    half_diag = 0.5 * math.hypot(shape[1] * spacing[1], shape[2] * spacing[2])
    w = _edge_width(4.0)
    ref = np.zeros(shape, dtype=np.float64)
    for k in range(n_beams):
        theta = math.radians(360.0 * k / n_beams + rng.uniform(0.0, 51.0))
        weight = rng.uniform(0.5, 1.0)
        n_rect = int(rng.integers(3, 9))
        dx, dy = math.cos(theta), math.sin(theta)
        lat = (-dy) * xx[None, :] + dx * yy[:, None]          # (ny, nx)
        depth = dx * xx[None, :] + dy * yy[:, None] + half_diag
        atten = np.exp(-0.0045 * depth)
        aperture = np.zeros(shape, dtype=np.float64)
        for _ in range(n_rect):
            su, sz = rng.uniform(10.0, 60.0, size=2)
            cu, cz = rng.uniform(-40.0, 40.0, size=2)
            fu = _soft_interval(lat, cu - su / 2, cu + su / 2, w)      # (ny, nx)
            fz = _soft_interval(zz, cz - sz / 2, cz + sz / 2, w)       # (nz,)
            np.maximum(aperture, fz[:, None, None] * fu[None, :, :], out=aperture)
        ref += weight * aperture * atten[None, :, :]
    ref /= ref.max()
    ev, meta = _perturb(ref, spacing, rng, hot_spot=hot_spot, axes=(zz, yy, xx))
    return DosePair(ref.astype(np.float32), ev.astype(np.float32), tuple(float(s) for s in spacing),
                    dict(meta, generator="3d-beams", seed=seed))


# Grid shapes of the workloads (slowest axis first) and spacings in mm.
CONFIG_SHAPES = {
    "2d_64x64_1mm": ((64, 64), (1.0, 1.0)),
    "3d_128x128x96_2.5mm": ((96, 128, 128), (2.5, 2.5, 2.5)),
    "3d_256x256x192_1.25mm": ((192, 256, 256), (1.25, 1.25, 1.25)),
}


def make_config_pair(config: str, seed: int) -> DosePair:
    shape, spacing = CONFIG_SHAPES[config]
    if len(shape) == 2:
        return make_pair_2d(seed, shape, spacing)
    return make_pair_3d(seed, shape, spacing)


@dataclass
class BatchSpec:
    """One pair of a mixed batch: the generator inputs and the gamma criteria."""
    seed: int
    shape: Tuple[int, ...]
    spacing: Tuple[float, ...]
    dd: float
    dta: float
    local: bool


def batch_specs(seed: int, n: int = 64, scale: float = 1.0):
    """The mixed batch: 2D or 3D with probability 1/2; 2D n x n nodes, n ~ U{128..200},
    h ~ U[1, 2] mm; 3D nx = ny ~ U{128..200}, nz ~ U{96..150}, h ~ U[1, 2] mm isotropic;
    criteria uniform over 3%/3mm, 2%/2mm, 1%/1mm; global or local with probability 1/2.
    ``scale`` shrinks every axis (small batches for tests).  Pair i uses seed seed + 1 + i."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        three = rng.uniform() < 0.5
        h = float(rng.uniform(1.0, 2.0))
        if three:
            nxy = int(rng.integers(128, 201))
            nz = int(rng.integers(96, 151))
            shape = (max(2, int(nz * scale)), max(2, int(nxy * scale)), max(2, int(nxy * scale)))
        else:
            m = int(rng.integers(128, 201))
            shape = (max(2, int(m * scale)), max(2, int(m * scale)))
        crit = int(rng.integers(0, 3))
        dd, dta = [(0.03, 3.0), (0.02, 2.0), (0.01, 1.0)][crit]
        local = bool(rng.uniform() < 0.5)
        out.append(BatchSpec(seed + 1 + i, shape, (h,) * len(shape), dd, dta, local))
    return out


def make_batch_pair(spec: "BatchSpec") -> DosePair:
    if len(spec.shape) == 2:
        return make_pair_2d(spec.seed, spec.shape, spec.spacing)
    return make_pair_3d(spec.seed, spec.shape, spec.spacing)
