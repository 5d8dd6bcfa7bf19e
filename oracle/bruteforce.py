"""Exhaustive gamma for tiny grids (test infrastructure only).

Independent of ``gamma_oracle.c``: it shares no code with it, enumerates EVERY face
(vertex, edge, triangle, tetrahedron) of the Kuhn triangulation of the whole grid,
applies no pruning and no initial bound, works in absolute (not reference-centred)
coordinates, and projects with Householder QR instead of the normal equations.

A face's affine-hull distance counts only when the orthogonal projection has all
barycentric weights >= 0 (it then lies in the face).  The minimum over the whole
triangulation is attained at such a projection on some face, so the minimum over the
accepted faces is the distance to the surface (Eq. (1) with the geometric method).
"""
from __future__ import annotations

from itertools import combinations, permutations
from typing import Sequence

import numpy as np


def kuhn_faces(shape: Sequence[int]):
    """All faces of the Kuhn triangulation of a grid, grouped by dimension.

    Returns a list ``faces[m]`` of int arrays (n_faces, m+1) of flat node indices.
    Every cube [q, q+1] is split into d! simplices q -> q+e_p1 -> ... -> q+(1,..,1);
    every non-empty vertex subset of every simplex is a face; duplicates are removed.
    """
    nd = len(shape)
    strides = np.array([int(np.prod(shape[i + 1:])) for i in range(nd)], dtype=np.int64)
    seen = [set() for _ in range(nd + 1)]
    for q in np.ndindex(*[n - 1 for n in shape]):
        q = np.array(q, dtype=np.int64)
        for perm in permutations(range(nd)):
            verts = [q.copy()]
            cur = q.copy()
            for ax in perm:
                cur = cur.copy()
                cur[ax] += 1
                verts.append(cur)
            lin = [int(np.dot(v, strides)) for v in verts]
            for m in range(nd + 1):
                for sub in combinations(lin, m + 1):
                    seen[m].add(tuple(sorted(sub)))
    return [np.array(sorted(s), dtype=np.int64).reshape(-1, m + 1) for m, s in enumerate(seen)]


def _node_coords(shape, spacing):
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) * h for n, h in zip(shape, spacing)],
                        indexing="ij")
    return np.stack([g.ravel() for g in grids], axis=1)      # (N, nd) in mm


def gamma_bruteforce(ref: np.ndarray, ev: np.ndarray, spacing: Sequence[float], dd: float,
                     dta: float, threshold: float = 0.1, local: bool = False) -> np.ndarray:
    """Gamma of every masked node; -1 elsewhere.  Meant for grids of a few hundred nodes."""
    ref = np.asarray(ref, dtype=np.float64)
    ev = np.asarray(ev, dtype=np.float64)
    shape = ref.shape
    faces = kuhn_faces(shape)
    xyz = _node_coords(shape, spacing) / dta                 # (N, nd), normalised
    rflat, eflat = ref.ravel(), ev.ravel()
    dmax = rflat.max()
    t = np.float64(np.float32(np.float64(np.float32(threshold)) * np.float64(np.float32(dmax))))
    mask = rflat >= t
    if local:
        mask &= rflat > 0
    out = np.full(rflat.size, -1.0)
    # QR of each face's edge matrix depends on dD; under global normalisation it is shared.
    cache = {}

    def factor(dD):
        key = float(dD)
        if key in cache:
            return cache[key]
        lifted = np.concatenate([xyz, (eflat / dD)[:, None]], axis=1)   # (N, nd+1)
        per_m = []
        for m, fm in enumerate(faces):
            base = lifted[fm[:, 0]]                                      # (F, A)
            if m == 0:
                per_m.append((base, None, None))
                continue
            V = np.stack([lifted[fm[:, i]] - base for i in range(1, m + 1)], axis=2)  # (F, A, m)
            Q, R = np.linalg.qr(V)                                       # Householder (LAPACK geqrf)
            per_m.append((base, Q, R))
        if not local:
            cache[key] = per_m
        return per_m

    for r in np.flatnonzero(mask):
        dD = dd * (rflat[r] if local else dmax)
        per_m = factor(dD)
        p = np.concatenate([xyz[r], [rflat[r] / dD]])
        best = np.inf
        for m, (base, Q, R) in enumerate(per_m):
            P = p[None, :] - base                                        # (F, A)
            if m == 0:
                best = min(best, float(np.min(np.einsum("fa,fa->f", P, P))))
                continue
            qtp = np.einsum("fam,fa->fm", Q, P)                          # (F, m)
            w = np.linalg.solve(R, qtp[..., None])[..., 0]               # weights of v1..vm
            w0 = 1.0 - w.sum(axis=1)
            inside = (w0 >= 0) & np.all(w >= 0, axis=1)
            if not np.any(inside):
                continue
            resid = P - np.einsum("fam,fm->fa", Q @ R, w)
            d2 = np.einsum("fa,fa->f", resid, resid)
            best = min(best, float(np.min(d2[inside])))
        out[r] = np.sqrt(best)
    return out.reshape(shape)
