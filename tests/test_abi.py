"""The C-ABI library loads and exports every symbol include/findpts.h
declares; host-side argument checks return FP_EINVAL / FP_ERANGE before any
device work (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

from paper_1811_04891_amd import findpts as fp

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "include", "findpts.h")


def _declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = "\n".join(l for l in src.splitlines() if not l.lstrip().startswith("#"))
    return sorted(set(re.findall(r"FP_API\s+[\w\s\*]*?\b(\w+)\s*\(", src)))


def test_header_declares_the_binding_symbols():
    assert sorted(fp.SYMBOLS) == _declared()


def test_library_exports_every_declared_symbol():
    L = fp.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_internal_symbols_hidden():
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", fp.LIB_PATH],
                         capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    assert exported == set(_declared())


def test_setup_argument_checks_without_gpu():
    L = fp.lib()
    h = C.c_void_p()
    x = C.c_void_p(16)  # never dereferenced: checks fail first
    assert L.findpts_setup(None, x, x, x, 1, 3, 1e-12, None, None, 10, 0, None) == fp.FP_EINVAL
    assert L.findpts_setup(C.byref(h), None, x, x, 1, 3, 1e-12, None, None, 10, 0, None) == fp.FP_EINVAL
    assert L.findpts_setup(C.byref(h), x, x, x, 1, 0, 1e-12, None, None, 10, 0, None) == fp.FP_ERANGE
    assert L.findpts_setup(C.byref(h), x, x, x, 1, 16, 1e-12, None, None, 10, 0, None) == fp.FP_ERANGE
    assert L.findpts_setup(C.byref(h), x, x, x, 0, 3, 1e-12, None, None, 10, 0, None) == fp.FP_EINVAL
    assert L.findpts_setup(C.byref(h), x, x, x, 1, 3, 0.0, None, None, 10, 0, None) == fp.FP_EINVAL
    assert L.findpts_setup(C.byref(h), x, x, x, 1, 3, 1e-12, None, None, 0, 0, None) == fp.FP_EINVAL
    assert L.findpts_setup(C.byref(h), x, x, x, 1, 3, 1e-12, None, None, 10, 7, None) == fp.FP_EINVAL
    assert L.fp_last_error().decode() != ""


def test_calls_on_null_handle():
    L = fp.lib()
    assert L.findpts(None, 1, None, None, None, None, None, None, None) == fp.FP_EINVAL
    assert L.findpts_eval(None, 1, None, None, None, 1, None, None, None) == fp.FP_EINVAL
    assert L.findpts_eval_noalloc(None, 1, None, None, None, 1, None, None, None) == fp.FP_EINVAL
    assert L.findpts_set_precision(None, 0) == fp.FP_EINVAL
    assert L.findpts_free(None) == fp.FP_OK
    assert L.fp_copy(C.c_void_p(8), C.c_void_p(16), 16, None) == fp.FP_EINVAL


def test_binding_rejects_cpu_tensors():
    import torch
    x = torch.zeros(27, dtype=torch.float64)
    with pytest.raises(ValueError):
        fp.findpts_setup(x, x, x, 2)


def test_serving_argument_checks_without_gpu():
    L = fp.lib()
    s = C.c_void_p()
    assert L.fps_create(None, 1 << 20, 2) == fp.FP_EINVAL
    assert L.fps_create(C.byref(s), 0, 2) == fp.FP_EINVAL
    assert L.fps_create(C.byref(s), 1 << 20, 0) == fp.FP_EINVAL
    assert L.fps_create(C.byref(s), 1 << 20, 17) == fp.FP_EINVAL
    mid = C.c_int()
    assert L.fps_add_mesh(None, None, None, 0, C.byref(mid)) == fp.FP_EINVAL
    t = C.c_longlong()
    assert L.fps_submit(None, 0, 1, None, None, 0, None, None, None, None, None, None,
                        C.byref(t)) == fp.FP_EINVAL
    assert L.fps_wait(None, 1, 0.0) == fp.FP_EINVAL
    d = C.c_double()
    assert L.fps_latency(None, C.byref(d), C.byref(d), C.byref(d), None, 0) == fp.FP_EINVAL
    assert L.fps_destroy(None) == fp.FP_OK


def test_2d_argument_checks_without_gpu():
    L = fp.lib()
    h = C.c_void_p()
    x = C.c_void_p(16)  # never dereferenced: checks fail first
    assert L.findpts2_setup(None, x, x, 1, 3, 1e-12, None, None, 10, None) == fp.FP_EINVAL
    assert L.findpts2_setup(C.byref(h), None, x, 1, 3, 1e-12, None, None, 10, None) == fp.FP_EINVAL
    assert L.findpts2_setup(C.byref(h), x, x, 1, 0, 1e-12, None, None, 10, None) == fp.FP_ERANGE
    assert L.findpts2_setup(C.byref(h), x, x, 1, 16, 1e-12, None, None, 10, None) == fp.FP_ERANGE
    assert L.findpts2_setup(C.byref(h), x, x, 0, 3, 1e-12, None, None, 10, None) == fp.FP_EINVAL
    assert L.findpts2_setup(C.byref(h), x, x, 1, 3, 1.0, None, None, 10, None) == fp.FP_EINVAL
    assert L.findpts2_setup(C.byref(h), x, x, 1, 3, 1e-12, None, None, 0, None) == fp.FP_EINVAL
    assert L.findpts2(None, 1, None, None, None, None, None, None, None) == fp.FP_EINVAL
    assert L.findpts2_eval(None, 1, None, None, None, 1, None, None, None) == fp.FP_EINVAL
    assert L.findpts2_free(None) == fp.FP_OK
    assert L.fp_last_error().decode() != ""
