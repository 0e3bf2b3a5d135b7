"""C-ABI contract checks that need no GPU: the library loads, exports every
function include/ctv.h declares, and rejects invalid arguments with
CTV_ERR_INVALID_ARG / CTV_ERR_WORKSPACE before any device work (all pointers
passed here are dummies that would fault if dereferenced)."""
import ctypes
import os
import re

import pytest

from paper_2109_05496_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ctv.h")
INVALID, WORKSPACE = -1, -2

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH), reason="libctv.so not built")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:ctv_status|int32_t|const char\*)\s+(\w+)\s*\(", text, flags=re.M)))


def test_header_and_binding_agree():
    assert header_functions() == sorted(_lib.EXPORTS)


def test_library_exports_every_header_symbol():
    L = ctypes.CDLL(_lib.LIB_PATH)
    for name in header_functions():
        assert hasattr(L, name), name
    assert _lib.lib().ctv_version() >= 100


def P(**kw):
    return _lib.make_params(**kw)


DUMMY = ctypes.c_void_p(0x1000)


def denoise_status(p, batch=1, m=8, n=8, lam=0.1, b=DUMMY, x=ctypes.c_void_p(0x2000), ws=DUMMY,
                   ws_bytes=1 << 40, state_in=None, k0=0, state_out=None, ckpt=0, saved=None):
    lams = (ctypes.c_float * batch)(*([lam] * batch))
    return _lib.lib().ctv_denoise(ctypes.byref(p), batch, m, n, b, lams, None, x, None, state_in, k0,
                                  state_out, ckpt, saved, ws, ws_bytes, None)


@pytest.mark.parametrize("bad", [
    dict(p=dict(kind="1i"), batch=0), dict(p=dict(kind="1i"), m=0), dict(p=dict(kind="1i"), n=-3),
    dict(p=dict(kind="1i"), lam=-0.1), dict(p=dict(kind="1i"), lam=float("nan")),
    dict(p=dict(kind="1i"), lam=float("inf")), dict(p=dict(kind="1i"), lam=1e-13),
    dict(p=dict(kind="1i"), lam=1e-40), dict(p=dict(kind="1i", iters=-1)),
    dict(p=dict(kind="2i", alpha=1.5)), dict(p=dict(kind="2i", alpha=-0.1)),
    dict(p=dict(kind="1i", fuse=17)), dict(p=dict(kind="1i"), b=None), dict(p=dict(kind="1i"), x=None),
    dict(p=dict(kind="1i"), ws=None), dict(p=dict(kind="1i"), k0=3),
    dict(p=dict(kind="1i", iters=30), ckpt=10, saved=None),
    dict(p=dict(kind="1i"), x=DUMMY),  # x aliases b
])
def test_invalid_arguments_rejected(bad):
    p = P(**bad.pop("p"))
    assert denoise_status(p, **bad) == INVALID
    assert _lib.lib().ctv_last_error()


def test_unknown_enums_and_struct_size():
    p = P()
    p.tv_kind = 7
    assert denoise_status(p) == INVALID
    p = P()
    p.constraint = 5
    assert denoise_status(p) == INVALID
    p = P()
    p.struct_size = 4
    assert denoise_status(p) == INVALID
    p = P()
    p.method = 2
    assert denoise_status(p) == INVALID
    with pytest.raises(ValueError):
        _lib.make_params(method="newton")


def test_workspace_too_small():
    p = P(iters=10)
    ws, sv = ctypes.c_size_t(), ctypes.c_size_t()
    assert _lib.lib().ctv_workspace_size(ctypes.byref(p), 2, 33, 40, 0, ctypes.byref(ws), ctypes.byref(sv)) == 0
    assert ws.value >= 2 * 2 * 33 * 40 * 16 * 2 and sv.value == 0
    assert denoise_status(p, batch=2, m=33, n=40, ws_bytes=ws.value - 1) == WORKSPACE


def test_checkpoint_storage_size():
    p = P(iters=50)
    ws, sv = ctypes.c_size_t(), ctypes.c_size_t()
    assert _lib.lib().ctv_workspace_size(ctypes.byref(p), 16, 512, 512, 10, ctypes.byref(ws), ctypes.byref(sv)) == 0
    # states at k = 10, 20, 30, 40 (k = 0 is the cold start)
    assert sv.value == 4 * 16 * 2 * 512 * 512 * 16


def test_python_wrapper_rejects_cpu_tensors():
    torch = pytest.importorskip("torch")
    import paper_2109_05496_amd as ctv
    with pytest.raises(TypeError):
        ctv.denoise(torch.zeros(4, 4, dtype=torch.complex64), 0.1)


def test_phase_retrieval_line_search_arguments_rejected():
    from paper_2109_05496_amd import api
    for kw in (dict(line_search=True, shrink=1.5), dict(line_search=True, shrink=0.0),
               dict(line_search=True, max_trials=0)):
        p, _keep = api._pr_params((1e-3,), 532e-9, 4e-6, 0.01, 0.5, 3, 5, "1i", 0.5, "modulus", 1, 1, 0,
                                  line_search=kw["line_search"], shrink=kw.get("shrink", 0.5),
                                  max_trials=kw.get("max_trials", 20))
        st = _lib.lib().pr_prox_grad(ctypes.byref(p), 8, 8, DUMMY, DUMMY, None, None, DUMMY, 1 << 40, None)
        assert st == INVALID, kw
        assert b"ls_" in _lib.lib().ctv_last_error()


def test_smallest_lambda_accepted():
    """lambda = 0 and lambda >= 1e-12 pass validation (the dummy pointers are
    never reached because the workspace check fails first); 0 < lambda < 1e-12,
    where 1/(8 lambda^2) overflows float32, is rejected."""
    p = P(iters=10)
    for lam in (0.0, 1e-12, 2e-12):
        assert denoise_status(p, lam=lam, ws_bytes=1) == WORKSPACE, lam
    for lam in (9e-13, 1e-20, 1e-45):
        assert denoise_status(p, lam=lam, ws_bytes=1) == INVALID, lam
        assert b"1e-12" in _lib.lib().ctv_last_error()


def test_flow_failure_hook_is_exported_and_host_only():
    assert _lib.lib().ctv_debug_flow_fail_waits(1) == 0
    assert _lib.lib().ctv_debug_flow_fail_waits(0) == 0


def test_noalloc_refuses_problems_above_its_scratch_before_device_work():
    p = P(iters=10)
    lams = (ctypes.c_float * 1)(0.1)
    st = _lib.lib().ctv_denoise_noalloc(ctypes.byref(p), 1, 2048, 2048, DUMMY, lams, None, ctypes.c_void_p(0x2000),
                                        None, None)
    assert st == WORKSPACE
    assert b"72" in _lib.lib().ctv_last_error() or b"workspace" in _lib.lib().ctv_last_error()
    assert _lib.lib().ctv_denoise_noalloc(ctypes.byref(p), 1, 8, 8, DUMMY, (ctypes.c_float * 1)(-1.0), None,
                                          ctypes.c_void_p(0x2000), None, None) == INVALID
