"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol include/apsp.h declares, and rejects bad arguments before touching
the device."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "apsp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("minplus_gemm", "apsp_fw", "apsp_rkleene", "apsp_batched", "apsp_validate"):
        assert required in names


def test_every_declared_symbol_is_exported(native):
    L = ctypes.CDLL(native.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name
    assert sorted(native.EXPORTS) == declared_functions()


def test_version_and_last_error(native):
    L = native.lib()
    assert b"gfx950" in L.apsp_version()
    assert isinstance(L.apsp_last_error(), bytes)


def _call_square(native, name, ctx, dt, n, ptr, ld, opts=None):
    L = native.lib()
    o = opts or native.make_opts()
    return getattr(L, name)(ctx, dt, n, ptr, ld, ctypes.byref(o), None)


@pytest.mark.parametrize("name", ["apsp_fw", "apsp_rkleene", "apsp_square", "apsp_solve", "apsp_closure"])
def test_argument_errors_before_any_device_call(native, name):
    fake = ctypes.c_void_p(0x1000)
    assert _call_square(native, name, None, 7, 4, fake, 4) == native.APSP_E_ARG
    assert "dtype" in native.last_error()
    assert _call_square(native, name, None, 0, -1, fake, 4) == native.APSP_E_ARG
    assert "negative" in native.last_error()
    assert _call_square(native, name, None, 0, 8, fake, 4) == native.APSP_E_ARG
    assert "ld" in native.last_error()
    assert _call_square(native, name, None, 0, 8, None, 8) == native.APSP_E_ARG
    assert "NULL" in native.last_error()
    bad = native.make_opts()
    bad.block = 96
    assert _call_square(native, name, None, 0, 8, fake, 8, bad) == native.APSP_E_ARG
    assert "block" in native.last_error()
    # valid arguments but no context
    assert _call_square(native, name, None, 0, 8, fake, 8) == native.APSP_E_ARG
    assert "context" in native.last_error()


def test_minplus_argument_errors(native):
    L = native.lib()
    o = native.make_opts()
    A, B, C = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x20000), ctypes.c_void_p(0x30000)
    f = L.minplus_gemm
    assert f(None, 0, -1, 2, 2, A, 2, B, 2, C, 2, ctypes.byref(o), None) == native.APSP_E_ARG
    assert f(None, 0, 2, 2, 2, A, 1, B, 2, C, 2, ctypes.byref(o), None) == native.APSP_E_ARG
    assert "lda" in native.last_error()
    assert f(None, 0, 2, 2, 2, A, 2, B, 1, C, 2, ctypes.byref(o), None) == native.APSP_E_ARG
    assert "ldb" in native.last_error()
    assert f(None, 0, 2, 2, 2, A, 2, B, 2, C, 1, ctypes.byref(o), None) == native.APSP_E_ARG
    assert "ldc" in native.last_error()
    # C overlapping A is rejected (the public product is out of place)
    assert f(None, 0, 4, 4, 4, A, 4, B, 4, ctypes.c_void_p(0x10008), 4, ctypes.byref(o), None) == native.APSP_E_ARG
    assert "overlap" in native.last_error()
    assert f(None, 0, 2, 2, 2, None, 2, B, 2, C, 2, ctypes.byref(o), None) == native.APSP_E_ARG
    assert f(None, 0, 2, 2, 2, A, 2, B, 2, C, 2, ctypes.byref(o), None) == native.APSP_E_ARG
    assert "context" in native.last_error()


def test_validate_argument_errors(native):
    L = native.lib()
    v = ctypes.c_int64(0)
    fake = ctypes.c_void_p(0x1000)
    assert L.apsp_validate(None, 0, 4, fake, 4, None, None) == native.APSP_E_ARG
    assert L.apsp_validate(None, 0, 4, fake, 2, None, ctypes.byref(v)) == native.APSP_E_ARG
    assert L.apsp_validate(None, 0, 4, fake, 4, None, ctypes.byref(v)) == native.APSP_E_ARG


def test_create_rejects_bad_arguments(native):
    L = native.lib()
    assert L.apsp_create(None, 0) == native.APSP_E_ARG
    c = ctypes.c_void_p()
    assert L.apsp_create(ctypes.byref(c), -1) == native.APSP_E_ARG
    assert L.apsp_destroy(None) == native.APSP_OK


def test_injected_create_failure_reports_hip_error(native):
    # forced from the host: no device call is made
    code = ("import ctypes, sys; sys.path.insert(0, %r);"
            "from paper_2310_03983_amd import apsp as a; c = ctypes.c_void_p();"
            "r = a.lib().apsp_create(ctypes.byref(c), 0);"
            "print(r, a.last_error())") % ROOT
    env = dict(os.environ, APSP_FAULT="create", HIP_VISIBLE_DEVICES="")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    status, msg = out.stdout.split(" ", 1)
    assert int(status) == native.APSP_E_HIP and "injected" in msg


def test_binding_rejects_host_tensors(native):
    import torch
    with pytest.raises(TypeError):
        native.apsp_fw(torch.zeros((4, 4), dtype=torch.int32))
    with pytest.raises(TypeError):
        native.apsp_fw(torch.zeros((4, 4), dtype=torch.float64))


def test_candidate_table(native):
    n = native.apsp_candidate_count()
    assert n >= 4
    algos = set()
    for i in range(n):
        o = native.apsp_candidate(i)
        assert o.algo in (1, 2, 3) and o.block in (0, 64, 128)
        assert o.flags in (0, native.FLAG_PACKED16)
        algos.add(o.algo)
    assert algos == {1, 2, 3}
    assert any(native.apsp_candidate(i).flags == native.FLAG_PACKED16 for i in range(n))
    with pytest.raises(native.ApspError):
        native.apsp_candidate(n)


def test_predecessors_argument_errors(native):
    L = native.lib()
    D, W, P = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x200000), ctypes.c_void_p(0x300000)
    f = L.apsp_predecessors
    assert f(None, 0, 4, D, 4, W, 4, P, 3, None) == native.APSP_E_ARG
    assert "ld" in native.last_error()
    assert f(None, 0, 4, D, 4, W, 4, ctypes.c_void_p(0x100010), 4, None) == native.APSP_E_ARG
    assert "overlap" in native.last_error()
    assert f(None, 0, 4, D, 4, W, 4, P, 4, None) == native.APSP_E_ARG
    assert "context" in native.last_error()


def test_packed16_option_is_checked_before_any_device_call(native):
    L = native.lib()
    fake = ctypes.c_void_p(0x1000)
    o = native.make_opts(packed16=True)
    # fp32 data: unsupported, for every solver
    for name in ("apsp_fw", "apsp_rkleene", "apsp_square", "apsp_solve"):
        assert _call_square(native, name, None, 1, 8, fake, 8, o) == native.APSP_E_UNSUPPORTED, name
        assert "int32" in native.last_error()
    # int32 data: accepted by the solvers (then the missing context is reported)
    for name in ("apsp_fw", "apsp_rkleene", "apsp_square", "apsp_solve"):
        assert _call_square(native, name, None, 0, 8, fake, 8, o) == native.APSP_E_ARG, name
        assert "context" in native.last_error()
    # entry points without the int32 redo reject it
    assert _call_square(native, "apsp_closure", None, 0, 8, fake, 8, o) == native.APSP_E_UNSUPPORTED
    A, B, C = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x20000), ctypes.c_void_p(0x30000)
    assert L.minplus_gemm(None, 0, 2, 2, 2, A, 2, B, 2, C, 2, ctypes.byref(o), None) == native.APSP_E_UNSUPPORTED
    assert "minplus_gemm" in native.last_error()
    n = (ctypes.c_int32 * 1)(4)
    assert L.apsp_batched(None, 0, 1, fake, fake, fake, n, ctypes.byref(o), None) == native.APSP_E_UNSUPPORTED
    runs, redone = ctypes.c_int64(), ctypes.c_int64()
    assert L.apsp_packed16_counts(None, ctypes.byref(runs), ctypes.byref(redone)) == native.APSP_E_ARG


def test_predecessors_ex_argument_errors(native):
    L = native.lib()
    D, W, P = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x200000), ctypes.c_void_p(0x300000)
    f = L.apsp_predecessors_ex
    assert f(None, 0, 4, D, 4, W, 4, P, 4, 3, None) == native.APSP_E_ARG
    assert "method" in native.last_error()
    assert f(None, 0, 4, D, 4, W, 4, P, 4, -1, None) == native.APSP_E_ARG
    big = 65536
    far = [ctypes.c_void_p(k << 36) for k in (1, 2, 3)]
    assert f(None, 0, big, far[0], big, far[1], big, far[2], big, native.PRED["sparse"], None) == \
        native.APSP_E_UNSUPPORTED
    assert f(None, 0, 4, D, 4, W, 4, P, 4, native.PRED["sparse"], None) == native.APSP_E_ARG
    assert "context" in native.last_error()


def _model_text(K=3, mu=(0.0, 1.0, 2.0, 3.0), sd=(1.0, 1.0, 0.5, 2.0), params=None, count=None):
    n = 4480 + 65 * K
    vals = params if params is not None else [0.001 * i for i in range(n)]
    lines = ["apsp-costmodel 1", f"K {K}", "in 4", "hidden 64",
             "mu " + " ".join(repr(float(x)) for x in mu), "sd " + " ".join(repr(float(x)) for x in sd),
             f"params {n if count is None else count}"] + [repr(float(v)) for v in vals]
    return "\n".join(lines) + "\n"


def test_costmodel_file_checks_before_the_context(native, tmp_path):
    """apsp_costmodel_load parses and checks the whole file before it looks at
    the context: malformed files fail with their reason even with a NULL
    context, a well-formed one then fails only on the NULL context."""
    L = native.lib()
    assert L.apsp_costmodel_load(None, None) == native.APSP_E_ARG and "NULL path" in native.last_error()
    assert L.apsp_costmodel_load(None, os.fsencode(str(tmp_path / "missing.txt"))) == native.APSP_E_ARG
    assert "cannot open" in native.last_error()
    good = _model_text()
    bad_cases = {
        "header": good.replace("apsp-costmodel 1", "apsp-costmodel 2"),
        "K missing or outside": good.replace("K 3", "K 65"),
        "layer sizes": good.replace("hidden 64", "hidden 32"),
        "sd not positive": _model_text(sd=(1.0, 0.0, 1.0, 1.0)),
        "mu / sd missing, not finite": _model_text(mu=(0.0, float("nan"), 0.0, 0.0)),
        "parameter count": _model_text(count=4480 + 65 * 3 - 1),
        "parameter missing": "\n".join(good.splitlines()[:-5]) + "\n",
        "not finite": _model_text(params=[0.0] * (4480 + 195 - 1) + [float("inf")]),
    }
    for reason, text in bad_cases.items():
        p = tmp_path / "m.txt"
        p.write_text(text)
        assert L.apsp_costmodel_load(None, os.fsencode(str(p))) == native.APSP_E_ARG, reason
        msg = native.last_error()
        assert "malformed" in msg and reason in msg, (reason, msg)
    p = tmp_path / "good.txt"
    p.write_text(good)
    assert L.apsp_costmodel_load(None, os.fsencode(str(p))) == native.APSP_E_ARG
    assert "context is NULL" in native.last_error()
    assert L.apsp_costmodel_save(None, os.fsencode(str(p))) == native.APSP_E_ARG
    assert L.apsp_costmodel_save(None, None) == native.APSP_E_ARG


def test_shipped_model_text_matches_its_json():
    """data/costmodel_mlp.txt (written by `autotune export`) holds exactly the
    binary32 values of data/costmodel_mlp.json."""
    import json
    import numpy as np
    data = os.path.join(ROOT, "paper_2310_03983_amd", "data")
    model = json.load(open(os.path.join(data, "costmodel_mlp.json")))
    lines = open(os.path.join(data, "costmodel_mlp.txt")).read().split("\n")
    assert lines[:4] == ["apsp-costmodel 1", f"K {model['K']}", "in 4", "hidden 64"]
    np.testing.assert_array_equal(np.float32(lines[4].split()[1:]), np.float32(model["mu"]))
    np.testing.assert_array_equal(np.float32(lines[5].split()[1:]), np.float32(model["sd"]))
    assert lines[6] == f"params {len(model['params'])}"
    np.testing.assert_array_equal(np.float32(lines[7:7 + len(model["params"])]), np.float32(model["params"]))


def test_fold_rate_argument_errors(native):
    L = native.lib()
    t, li = ctypes.c_double(), ctypes.c_double()
    assert L.apsp_measure_fold_rate(None, 3, None, ctypes.byref(t), ctypes.byref(li)) == native.APSP_E_ARG
    assert "fold" in native.last_error()
    assert L.apsp_measure_fold_rate(None, 0, None, None, ctypes.byref(li)) == native.APSP_E_ARG
    assert L.apsp_measure_fold_rate(None, 0, None, ctypes.byref(t), ctypes.byref(li)) == native.APSP_E_ARG
    assert "context is NULL" in native.last_error()
