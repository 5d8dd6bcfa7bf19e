"""Planted mistakes in the gamma oracle each fail a pin.

Each mutant is a copy of ``oracle/gamma_oracle.c`` with one plausible mistake written in
(a text substitution of a line that must occur exactly once), compiled to a library of its
own and put in place of the oracle for the pins below:

* the exhaustive search of ``oracle.bruteforce`` on tiny 2D and 3D grids (smooth and rough
  fields, global and local normalisation, anisotropic spacing);
* the closed forms: identical doses give 0; a flat offset gives |delta| / dD; a shifted
  linear ramp gives the point-to-plane distance |a.s| / sqrt(dD^2 + DTA^2 |a|^2).

The unmutated source passes the same pins, so each failure is the planted mistake's.
"""
import ctypes as C
import math
import os
import subprocess

import numpy as np
import pytest

from oracle import core
from oracle.bruteforce import gamma_bruteforce
from dosegen import make_pair_2d, make_pair_3d

SRC = os.path.join(os.path.dirname(core.__file__), "gamma_oracle.c")

# (name, text in the oracle, replacement)
MUTATIONS = [
    ("early break: the key compared with gamma squared",
     "if (tab[e].key >= g) break;", "if (tab[e].key * tab[e].key >= g) break;"),
    ("ignored weight: the base vertex's barycentric weight never tested",
     "for (int i = 0; i <= m; ++i) any_neg |= (w[i] < 0.0);",
     "for (int i = 0; i < m; ++i) any_neg |= (w[i] < 0.0);"),
    ("off-by-one cell range: the last cell of every axis skipped",
     "if (q[i] < 0 || q[i] > n[i] - 2) inside = 0;", "if (q[i] < 0 || q[i] > n[i] - 3) inside = 0;"),
    ("wrong key: the distance to the cell at a negative offset taken from its far corner",
     "else if (a[i] < -1) g = (double)(-a[i] - 1);", "else if (a[i] < 0) g = (double)(-a[i]);"),
    ("sign: the cell's corners placed on the wrong side of its lower corner",
     "corner[b][i] = (double)(tab[e].a[i] + bit) * pb->spacing[i] / pb->dta;",
     "corner[b][i] = (double)(tab[e].a[i] - bit) * pb->spacing[i] / pb->dta;"),
    ("dropped term: the Gram matrix without the dose component",
     "for (int a = 0; a < amb; ++a) s += V[a][i] * V[a][j];",
     "for (int a = 0; a < amb - 1; ++a) s += V[a][i] * V[a][j];"),
    ("transposed operand: the forward substitution reads L transposed",
     "for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];", "for (int k = 0; k < i; ++k) s -= L[k][i] * y[k];"),
    ("local normalisation: the search uses the global dD",
     "double dD = pb->local ? pb->dd * ref[r] : dD_global;\n            double g0 = fabs(ev[r] - ref[r]) / dD;",
     "double dD = dD_global;\n            double g0 = fabs(ev[r] - ref[r]) / dD;"),
]


def _rough_pair(seed, shape, amp=0.3):
    rng = np.random.default_rng(seed)
    ref = rng.uniform(0.2, 1.0, size=shape) + amp * rng.standard_normal(shape)
    ev = ref + amp * rng.standard_normal(shape)
    ref = ref / ref.max()
    return ref.astype(np.float32), ev.astype(np.float32)


def _brute(ref, ev, spacing, dd, dta, thr, local):
    def check():
        o = core.gamma(ref, ev, spacing, dd, dta, thr, local)
        m = o.gamma >= 0
        return bool(m.any()) and np.array_equal(m, b >= 0) and float(np.abs(o.gamma[m] - b[m]).max()) <= 1e-10
    b = gamma_bruteforce(ref, ev, spacing, dd, dta, thr, local)
    return check


def _identical():
    rng = np.random.default_rng(1)
    ref = rng.uniform(0, 1, size=(6, 7, 8)).astype(np.float32)
    o = core.gamma(ref, ref, (1.0, 2.0, 3.0), 0.03, 3.0, 0.1)
    m = o.gamma >= 0
    return bool(m.any()) and bool(np.all(o.gamma[m] == 0.0))


def _flat(local):
    ref = np.full((5, 6, 7), 0.75)
    o = core.gamma(ref, ref + 0.025, (2.5, 1.0, 2.0), 0.03, 3.0, 0.1, local)
    return bool(np.allclose(o.gamma, 0.025 / (0.03 * 0.75), rtol=1e-12, atol=1e-12))


def _ramp():
    shape, spacing = (9, 10, 11), (2.0, 1.5, 1.0)
    a, s, dd, dta = np.array([0.01, -0.02, 0.015]), np.array([0.7, -0.4, 1.1]), 0.03, 3.0
    X = np.meshgrid(*[np.arange(n) * h for n, h in zip(shape, spacing)], indexing="ij")
    lin = sum(ai * xi for ai, xi in zip(a, X))
    ref, ev = 0.5 + lin, 0.5 + lin - float(a @ s)
    dD = dd * ref.max()
    expect = abs(float(a @ s)) / math.sqrt(dD ** 2 + dta ** 2 * float(a @ a))
    o = core.gamma(ref, ev, spacing, dd, dta, 0.0)
    inner = tuple(slice(3, n - 3) for n in shape)
    return bool(np.allclose(o.gamma[inner], expect, rtol=1e-9, atol=1e-12))


@pytest.fixture(scope="module")
def pins():
    p2 = make_pair_2d(0, shape=(20, 18), spacing=(1.0, 1.5))
    p3 = make_pair_3d(5, shape=(7, 8, 9), spacing=(2.5, 2.0, 2.0))
    r2, e2 = _rough_pair(3, (11, 13))
    r3, e3 = _rough_pair(6, (5, 6, 7))
    return {
        "brute 2D smooth global": _brute(p2.ref, p2.eval, p2.spacing, 0.01, 1.0, 0.1, False),
        "brute 2D rough local": _brute(r2, e2, (2.0, 0.7), 0.05, 2.0, 0.0, True),
        "brute 3D smooth 1%/1mm": _brute(p3.ref, p3.eval, p3.spacing, 0.01, 1.0, 0.0, False),
        "brute 3D smooth local": _brute(p3.ref, p3.eval, p3.spacing, 0.02, 2.0, 0.0, True),
        "brute 3D rough": _brute(r3, e3, (1.5, 0.8, 1.2), 0.05, 2.0, 0.0, False),
        "identical doses": _identical,
        "flat offset global": lambda: _flat(False),
        "flat offset local": lambda: _flat(True),
        "shifted ramp": _ramp,
    }


def _failing(pins):
    return [name for name, check in pins.items() if not check()]


def _build(src_text, path):
    c_path = path + ".c"
    with open(c_path, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", path, c_path, "-lm"])
    return core.configure(C.CDLL(path))


def test_unmutated_oracle_passes_every_pin(pins):
    assert _failing(pins) == []


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0].split(":")[0] for m in MUTATIONS])
def test_planted_mistake_fails_a_pin(pins, tmp_path, monkeypatch, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"the line to mutate is not unique in the oracle: {old}"
    lib = _build(src.replace(old, new), str(tmp_path / "libmutant.so"))
    monkeypatch.setattr(core, "_lib", lib)
    failing = _failing(pins)
    assert failing, f"no pin catches the planted mistake ({name})"
