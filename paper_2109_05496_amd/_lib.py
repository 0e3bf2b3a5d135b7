"""ctypes loader and signatures for ``libctv.so`` (the C ABI in include/ctv.h).

Loading fails loudly when the library has not been built: there is no CPU
fallback anywhere in the product path.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libctv.so")

CTV_OK = 0
KINDS = {"1i": 0, "1a": 1, "2i": 2, "2a": 3}
CONSTRAINTS = {"none": 0, "modulus": 1}
METHODS = {"fgp": 0, "gp": 1}
SCHEDULES = {"auto": 0, "steps": 1, "flow": 2}

c_f = ctypes.c_float
c_d = ctypes.c_double
c_i32 = ctypes.c_int32
c_u32 = ctypes.c_uint32
c_i64 = ctypes.c_int64
c_sz = ctypes.c_size_t
c_vp = ctypes.c_void_p
c_psz = ctypes.POINTER(ctypes.c_size_t)


class CtvError(RuntimeError):
    """A C-ABI call returned a non-zero status."""

    def __init__(self, func, status, msg):
        super().__init__(f"{func} failed with status {status}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("struct_size", c_u32), ("tv_kind", c_i32), ("alpha", c_f),
                ("constraint", c_i32), ("iters", c_i32), ("fuse", c_i32), ("tile_waves", c_i32),
                ("tile_rows", c_i32), ("method", c_i32), ("schedule", c_i32)]


class ImageDesc(ctypes.Structure):
    _fields_ = [("offset", c_i64), ("m", c_i32), ("n", c_i32), ("lam", c_f), ("tv_kind", c_i32),
                ("alpha", c_f), ("iters", c_i32), ("support_offset", c_i64)]


class PrParams(ctypes.Structure):
    _fields_ = [("struct_size", c_u32), ("num_meas", c_i32), ("distances_host", ctypes.POINTER(c_d)),
                ("wavelength", c_d), ("pixel", c_d), ("tau", c_f), ("gamma", c_f),
                ("outer_iters", c_i32), ("inner", Params), ("init_backprop", c_i32),
                ("accelerate", c_i32), ("line_search", c_i32), ("ls_shrink", c_f), ("ls_max_trials", c_i32),
                ("warm_start", c_i32)]


class Tuning(ctypes.Structure):
    _fields_ = [("fuse", c_i32), ("tile_waves", c_i32), ("tile_rows", c_i32), ("ms", c_f)]


_SIGS = {
    "ctv_version": (c_i32, []),
    "ctv_last_error": (ctypes.c_char_p, []),
    "ctv_debug_flow_fail_waits": (c_i32, [c_i32]),
    "ctv_tiling": (c_i32, [ctypes.POINTER(Params), c_i32, c_i32, c_i32, ctypes.POINTER(c_i32),
                           ctypes.POINTER(c_i32), ctypes.POINTER(c_i32), ctypes.POINTER(c_i32)]),
    "ctv_workspace_size": (c_i32, [ctypes.POINTER(Params), c_i32, c_i32, c_i32, c_i32, c_psz, c_psz]),
    "ctv_denoise": (c_i32, [ctypes.POINTER(Params), c_i32, c_i32, c_i32, c_vp, ctypes.POINTER(c_f), c_vp,
                            c_vp, c_vp, c_vp, c_i32, c_vp, c_i32, c_vp, c_vp, c_sz, c_vp]),
    "ctv_denoise_noalloc": (c_i32, [ctypes.POINTER(Params), c_i32, c_i32, c_i32, c_vp, ctypes.POINTER(c_f), c_vp,
                                    c_vp, c_vp, c_vp]),
    "ctv_batched_plan_create": (c_i32, [ctypes.POINTER(ImageDesc), c_i32, ctypes.POINTER(Params),
                                        ctypes.POINTER(c_vp)]),
    "ctv_batched_workspace_size": (c_i32, [c_vp, c_psz]),
    "ctv_denoise_batched": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "ctv_batched_plan_destroy": (c_i32, [c_vp]),
    "ctv_batched_plan_tiling": (c_i32, [c_vp, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32), ctypes.POINTER(c_i32)]),
    "ctv_autotune": (c_i32, [ctypes.POINTER(Params), c_i32, c_i32, c_i32, c_vp, ctypes.POINTER(c_f), c_vp, c_vp,
                             c_vp, c_sz, c_i32, ctypes.POINTER(Tuning), c_i32, ctypes.POINTER(c_i32),
                             ctypes.POINTER(Tuning), c_vp]),
    "ctv_batched_autotune": (c_i32, [ctypes.POINTER(ImageDesc), c_i32, ctypes.POINTER(Params), c_vp, c_vp, c_vp,
                                     c_vp, c_sz, c_i32, ctypes.POINTER(Tuning), c_i32, ctypes.POINTER(c_i32),
                                     ctypes.POINTER(Tuning), c_vp]),
    "ctv_tune_lookup": (c_i32, [ctypes.POINTER(Params), c_i32, c_i32, c_i32, ctypes.POINTER(c_i32),
                                ctypes.POINTER(Tuning)]),
    "ctv_batched_tune_lookup": (c_i32, [ctypes.POINTER(ImageDesc), c_i32, ctypes.POINTER(Params),
                                        ctypes.POINTER(c_i32), ctypes.POINTER(Tuning)]),
    "ctv_tune_cache_save": (c_i32, [ctypes.c_char_p]),
    "ctv_tune_cache_load": (c_i32, [ctypes.c_char_p]),
    "ctv_tune_cache_clear": (c_i32, []),
    "ctv_tune_cache_size": (c_i32, []),
    "ctv_backward_workspace_size": (c_i32, [ctypes.POINTER(Params), c_i32, c_i32, c_i32, c_i32, c_psz]),
    "ctv_denoise_backward": (c_i32, [ctypes.POINTER(Params), c_i32, c_i32, c_i32, c_vp, ctypes.POINTER(c_f),
                                     c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "pr_workspace_size": (c_i32, [ctypes.POINTER(PrParams), c_i32, c_i32, c_psz]),
    "pr_prox_grad": (c_i32, [ctypes.POINTER(PrParams), c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "pr_ip": (c_i32, [ctypes.POINTER(PrParams), c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "ctv_fft2_workspace_size": (c_i32, [c_i32, c_i32, c_i32, c_psz]),
    "ctv_fft2": (c_i32, [c_i32, c_i32, c_i32, c_vp, c_vp, c_i32, c_vp, c_sz, c_vp]),
    "pr_forward": (c_i32, [ctypes.POINTER(PrParams), c_i32, c_i32, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "pr_gradient": (c_i32, [ctypes.POINTER(PrParams), c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
}

EXPORTS = tuple(_SIGS)

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2109_05496_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(name, status):
    if status != CTV_OK:
        msg = lib().ctv_last_error()
        raise CtvError(name, status, msg.decode() if msg else "")


def call(name, *args):
    check(name, getattr(lib(), name)(*args))


def make_params(kind="1i", alpha=0.5, constraint="modulus", iters=100, fuse=0, tile=(0, 0), method="fgp",
                schedule="auto"):
    if method not in METHODS:
        raise ValueError(f"unknown method {method!r}")
    if schedule not in SCHEDULES:
        raise ValueError(f"unknown schedule {schedule!r}")
    if kind not in KINDS:
        raise ValueError(f"unknown TV kind {kind!r}")
    if constraint not in CONSTRAINTS:
        raise ValueError(f"unknown constraint {constraint!r}")
    return Params(ctypes.sizeof(Params), KINDS[kind], float(alpha), CONSTRAINTS[constraint], int(iters),
                  int(fuse), int(tile[0]), int(tile[1]), METHODS[method], SCHEDULES[schedule])
