"""The C ABI library: it loads, exports every function include/gammax.h declares, and
rejects bad arguments on the host before touching a device (no GPU needed)."""
import ctypes as C
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gammax.h")


@pytest.fixture(scope="module")
def abi():
    lib_path = os.path.join(ROOT, "paper_1012_1900_amd", "lib", "libgammax.so")
    if not os.path.exists(lib_path):
        from paper_1012_1900_amd import _build
        _build.build()
    from paper_1012_1900_amd import _abi
    return _abi


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+char\s*\*|gammax_status_t|void)\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["gamma_map", "gammax_map", "gammax_ctx_create", "gammax_ctx_destroy",
                 "gammax_sort_pairs", "gammax_build_table", "gammax_pass_count",
                 "gammax_status_string", "gammax_last_error", "gammax_options_default",
                 "gammax_model_create", "gammax_model_destroy", "gammax_model_get_params",
                 "gammax_model_features", "gammax_model_predict", "gammax_model_forward",
                 "gammax_model_train_step", "gammax_model_last_error", "gammax_model_predict_nodes",
                 "gammax_batch", "gammax_tune_save", "gammax_tune_load", "gammax_map_async",
                 "gammax_map_wait", "gammax_map_many", "gammax_model_predict_nodes_pooled", "gammax_map_grids",
                 "gammax_model_save", "gammax_model_load"]:
        assert must in names


def test_library_exports_every_declared_symbol(abi):
    lib = abi.raw_library()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_options_defaults(abi):
    o = abi.default_options()
    assert o.sort_mode == abi.SORT_NONE
    assert o.precision == abi.PREC_GUARDED
    assert o.cond_threshold == 1e6
    assert o.timing == 0 and o.tail_lanes == 0 and o.cell_lanes == 0 and list(o.reserved) == [0]
    assert o.autotune == 0 and o.cnn_pool == 0 and o.projection == 0 and o.order_key is None
    assert o.radius_mode == abi.RADIUS_PLAIN and not o.model and o.radius_factor == 1.1


def test_options_given_order(abi):
    o = abi.make_options(sort="given", order_key=0x7f0000001000)
    assert o.sort_mode == abi.SORT_GIVEN == 4 and o.order_key == 0x7f0000001000
    assert abi.make_options(sort="dd").order_key is None


def test_status_strings(abi):
    for st in range(0, -10, -1):
        s = abi.status_string(st)
        assert s and s != "unknown status"
    assert abi.status_string(-99) == "unknown status"


def _flat(abi, ndim=2, shape=(16, 16), spacing=(1.0, 1.0), dd=0.03, dta=3.0, thr=0.1, norm=0,
          ptr=1):
    lib = abi.raw_library()
    sh = (C.c_int64 * 3)(*(list(shape) + [0] * (3 - len(shape))))
    sp = (C.c_double * 3)(*(list(spacing) + [0.0] * (3 - len(spacing))))
    p = C.c_void_p(ptr) if ptr else None
    return lib.gamma_map(p, p, ndim, sh, sp, dd, dta, thr, norm, p, None, None)


@pytest.mark.parametrize("kw,expect", [
    (dict(ptr=0), -1),
    (dict(ndim=4), -2),
    (dict(ndim=1), -2),
    (dict(shape=(1, 16)), -2),
    (dict(ndim=3, shape=(2, 2, 1)), -2),
    (dict(ndim=3, shape=(2048, 2048, 2048), spacing=(1, 1, 1)), -2),
    (dict(spacing=(0.0, 1.0)), -3),
    (dict(spacing=(1.0, -2.0)), -3),
    (dict(spacing=(1.0, math.inf)), -3),
    (dict(dd=0.0), -3),
    (dict(dd=math.nan), -3),
    (dict(dta=-1.0), -3),
    (dict(thr=1.0), -3),
    (dict(thr=-0.01), -3),
    (dict(norm=2), -3),
])
def test_host_argument_checks(abi, kw, expect):
    assert _flat(abi, **kw) == expect


def test_null_context(abi):
    lib = abi.raw_library()
    r = abi.Result()
    p = abi.make_problem((8, 8), (1.0, 1.0), 0.03, 3.0, 0.1, False)
    assert lib.gammax_map(None, C.byref(p), None, None, None, None, C.byref(r), None) == abi.E_NULL
    t = C.c_uint64(7)
    assert lib.gammax_map_async(None, C.byref(p), None, None, None, None, C.byref(t), None) == abi.E_NULL
    assert lib.gammax_map_wait(None, 1, C.byref(r)) == abi.E_NULL
    assert lib.gammax_map_many(None, 1, None, None, None, None, None, None, None) == abi.E_NULL
    assert lib.gammax_sort_pairs(None, None, None, 0, None) == abi.E_NULL
    assert lib.gammax_pass_count(None, None, 0, None, None) == abi.E_NULL
    assert lib.gammax_ctx_destroy(None) == abi.OK


def test_null_model(abi):
    lib = abi.raw_library()
    h = C.c_void_p()
    crop = (C.c_int64 * 3)(8, 8, 8)
    hp = abi.Adam(1e-3, 0.9, 0.999, 1e-8)
    assert lib.gammax_model_create(0, None, C.byref(h)) == abi.E_NULL
    assert lib.gammax_model_destroy(None) == abi.OK
    assert lib.gammax_model_get_params(None, None, None) == abi.E_NULL
    assert lib.gammax_model_forward(None, 1, crop, None, None, None) == abi.E_NULL
    assert lib.gammax_model_train_step(None, 1, crop, None, None, C.byref(hp), None, None) == abi.E_NULL
    assert lib.gammax_model_predict(None, None, None, None, None, None, None) == abi.E_NULL
    assert lib.gammax_model_features(None, None, None, None, None, None) == abi.E_NULL
    assert lib.gammax_model_last_error(None) == b""
    assert lib.gammax_model_save(None, b"/tmp/x") == abi.E_NULL
    assert lib.gammax_model_load(0, None, C.byref(h)) == abi.E_NULL
    assert lib.gammax_model_load(0, b"/tmp/x", None) == abi.E_NULL


def test_model_file_checks_before_any_device_call(abi, tmp_path):
    """gammax_model_load refuses a missing file, another format or version, another
    parameter count, short or long data and non-finite values (GAMMAX_E_MODEL) before it
    touches a device."""
    import numpy as np
    lib = abi.raw_library()
    n = abi.MODEL_NPARAM

    def head(**kw):
        d = {"format": "gammax-model", "version": 1, "nparam": n, "adam_step": 4}
        d.update(kw)
        return ("{" + ", ".join(f'"{k}": ' + (f'"{v}"' if isinstance(v, str) else str(v)) for k, v in d.items())
                + ', "arrays": ["params", "adam_m", "adam_v"], "dtype": "float32-le"}\n').encode()

    data = np.zeros(3 * n, dtype="<f4").tobytes()
    nan = np.zeros(3 * n, dtype="<f4")
    nan[n + 5] = np.nan
    cases = {"missing": None, "format": head(format="other") + data, "version": head(version=2) + data,
             "nparam": head(nparam=n - 1) + data, "short": head() + data[:-4], "long": head() + data + b"\0",
             "nonfinite": head() + nan.tobytes(), "step": head(adam_step=-1) + data}
    for name, raw in cases.items():
        path = tmp_path / f"{name}.ckpt"
        if raw is not None:
            path.write_bytes(raw)
        h = C.c_void_p()
        assert lib.gammax_model_load(0, str(path).encode(), C.byref(h)) == abi.E_MODEL, name
        assert not h.value


def test_struct_layouts_match_the_header(abi, tmp_path):
    """ctypes mirrors of the C structs have the C compiler's sizes and offsets."""
    import subprocess
    structs = {"gammax_problem_t": abi.Problem, "gammax_options_t": abi.Options,
               "gammax_result_t": abi.Result, "gammax_adam_t": abi.Adam}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "gammax.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f in py._fields_:
            assert got[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])
