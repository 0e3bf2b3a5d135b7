"""Python API over the C ABI. Argument marshalling only: tensors must already be
on the GPU; every step of the solver runs in the HIP library."""
import ctypes

import torch

from . import _lib
from ._lib import call, make_params


def _stream(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _require_cuda(t, name, dtype=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _out_like(out, b):
    """The output tensor: ``out`` (complex64, contiguous, b's shape) or a new one."""
    if out is None:
        return torch.empty_like(b)
    _require_cuda(out, "out", torch.complex64)
    if tuple(out.shape) != tuple(b.shape):
        raise ValueError(f"out must have shape {tuple(b.shape)}, got {tuple(out.shape)}")
    return out


def _lams(lam, batch):
    if isinstance(lam, torch.Tensor):
        lam = lam.detach().cpu().reshape(-1).tolist()
    elif isinstance(lam, (int, float)):
        lam = [float(lam)] * batch
    lam = [float(v) for v in lam]
    if len(lam) == 1 and batch > 1:
        lam = lam * batch
    if len(lam) != batch:
        raise ValueError("lambda must be a scalar or have one value per image")
    return (ctypes.c_float * batch)(*lam)


def tiling(fuse=0, iters=100, m=2048, n=2048, batch=1, tile=(0, 0), detail=False, kind="1i",
           constraint="modulus", method="fgp"):
    """(iterations fused per launch, tile region rows) that ctv_denoise uses;
    with detail=True also (tile_waves, rows_per_thread)."""
    p = make_params(kind, 0.5, constraint, iters, fuse, tile, method)
    t, r, w, rp = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    call("ctv_tiling", ctypes.byref(p), batch, m, n, ctypes.byref(t), ctypes.byref(r), ctypes.byref(w),
         ctypes.byref(rp))
    return (t.value, r.value, w.value, rp.value) if detail else (t.value, r.value)


def workspace_size(m, n, batch=1, kind="1i", alpha=0.5, constraint="modulus", iters=100, fuse=0,
                   ckpt_every=0, method="fgp"):
    """(workspace bytes, checkpoint bytes) for ``denoise``."""
    p = make_params(kind, alpha, constraint, iters, fuse, method=method)
    ws, sv = ctypes.c_size_t(), ctypes.c_size_t()
    call("ctv_workspace_size", ctypes.byref(p), batch, m, n, ckpt_every, ctypes.byref(ws), ctypes.byref(sv))
    return ws.value, sv.value


def denoise(b, lam, kind="1i", alpha=0.5, constraint="modulus", support=None, iters=100, fuse=0,
            gap=False, state=None, k0=0, return_state=False, ckpt_every=0, saved=None, out=None,
            workspace=None, tile=(0, 0), method="fgp", schedule="auto"):
    """K FGP iterations (Algorithm 2) + Eq. (18) on the GPU.

    b: complex64 CUDA tensor [m, n] or [B, m, n]. lam: float or B floats.
    support: uint8 [m, n] or None. method: "fgp" (Algorithm 2) or "gp" (the
    unaccelerated iteration of Eq. 21). schedule: "auto", "steps" (one launch
    per fused step) or "flow" (one persistent launch); results are identical.
    Returns x (and the duality gap as a float64 tensor [B] when gap=True, and
    the dual state when return_state=True).
    """
    _require_cuda(b, "b", torch.complex64)
    squeeze = b.dim() == 2
    bb = b.unsqueeze(0) if squeeze else b
    B, m, n = bb.shape
    dev = bb.device
    p = make_params(kind, alpha, constraint, iters, fuse, tile, method, schedule)
    if support is not None:
        _require_cuda(support, "support", torch.uint8)
        if tuple(support.shape) != (m, n):
            raise ValueError("support must be [m, n]")
    x = _out_like(out, b)
    ws_bytes, sv_bytes = workspace_size(m, n, B, kind, alpha, constraint, iters, fuse, ckpt_every, method)
    ws = workspace if workspace is not None else torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    g = torch.empty(B, dtype=torch.float64, device=dev) if gap else None
    st_out = torch.empty((B, 2, m, n, 4), dtype=torch.float32, device=dev) if return_state else None
    if state is not None:
        _require_cuda(state, "state", torch.float32)
    if ckpt_every and saved is None and sv_bytes:
        saved = torch.empty(sv_bytes // 4, dtype=torch.float32, device=dev)
    call("ctv_denoise", ctypes.byref(p), B, m, n, _ptr(bb), _lams(lam, B), _ptr(support), _ptr(x),
         _ptr(g), _ptr(state), int(k0), _ptr(st_out), int(ckpt_every), _ptr(saved), _ptr(ws),
         ws.numel(), _stream(dev))
    res = [x]
    if gap:
        res.append(g)
    if return_state:
        res.append(st_out)
    if ckpt_every:
        res.append(saved)
    return res[0] if len(res) == 1 else tuple(res)


def denoise_backward(b, lam, grad_x, saved, kind="1i", alpha=0.5, constraint="modulus", support=None,
                     iters=100, fuse=0, ckpt_every=10, method="fgp"):
    """Reverse pass of the K-step map; returns (grad_b, grad_lambda[B])."""
    _require_cuda(b, "b", torch.complex64)
    _require_cuda(grad_x, "grad_x", torch.complex64)
    squeeze = b.dim() == 2
    bb = b.unsqueeze(0) if squeeze else b
    gx = grad_x.unsqueeze(0) if squeeze else grad_x
    B, m, n = bb.shape
    dev = bb.device
    p = make_params(kind, alpha, constraint, iters, fuse, method=method)
    ws_bytes = ctypes.c_size_t()
    call("ctv_backward_workspace_size", ctypes.byref(p), B, m, n, ckpt_every, ctypes.byref(ws_bytes))
    ws = torch.empty(ws_bytes.value, dtype=torch.uint8, device=dev)
    gb = torch.empty_like(bb)
    gl = torch.empty(B, dtype=torch.float32, device=dev)
    call("ctv_denoise_backward", ctypes.byref(p), B, m, n, _ptr(bb), _lams(lam, B), _ptr(support),
         int(ckpt_every), _ptr(saved), _ptr(gx.contiguous()), _ptr(gb), _ptr(gl), _ptr(ws), ws.numel(),
         _stream(dev))
    return (gb[0] if squeeze else gb), gl


class CTVDenoise(torch.autograd.Function):
    """x = FGP_K(b, lambda) with gradients for b (complex64) and lambda.

    apply(b, lam, kind, alpha, constraint, support, iters, ckpt_every, fuse, method).
    lam may be a Python float (no gradient) or a float32 tensor of shape [] or
    [B]; a scalar tensor receives the sum of the per-image gradients.
    """

    @staticmethod
    def forward(ctx, b, lam, kind="1i", alpha=0.5, constraint="modulus", support=None, iters=50,
                ckpt_every=10, fuse=0, method="fgp"):
        lam_vals = lam.detach() if isinstance(lam, torch.Tensor) else lam
        x, saved = denoise(b, lam_vals, kind, alpha, constraint, support, iters, fuse,
                           ckpt_every=ckpt_every, method=method)
        ctx.save_for_backward(b, saved)
        ctx.lam = lam_vals.cpu().reshape(-1).tolist() if isinstance(lam_vals, torch.Tensor) else lam_vals
        ctx.lam_shape = lam.shape if isinstance(lam, torch.Tensor) else None
        ctx.lam_meta = (lam.device, lam.dtype) if isinstance(lam, torch.Tensor) else None
        ctx.cfg = (kind, alpha, constraint, support, iters, fuse, ckpt_every, method)
        return x

    @staticmethod
    def backward(ctx, grad_x):
        b, saved = ctx.saved_tensors
        kind, alpha, constraint, support, iters, fuse, ckpt_every, method = ctx.cfg
        gb, gl = denoise_backward(b, ctx.lam, grad_x.contiguous(), saved, kind, alpha, constraint, support,
                                  iters, fuse, ckpt_every, method)
        glam = None
        if ctx.lam_shape is not None:
            glam = gl.sum().reshape(ctx.lam_shape) if len(ctx.lam_shape) == 0 or ctx.lam_shape.numel() == 1 \
                else gl.reshape(ctx.lam_shape)
            glam = glam.to(device=ctx.lam_meta[0], dtype=ctx.lam_meta[1])
        return gb, glam, None, None, None, None, None, None, None, None


def _image_descs(images):
    """ctv_image_desc array for images packed back to back in the order given,
    with (offsets, support offsets, shapes, total pixels, support bytes)."""
    descs = (_lib.ImageDesc * len(images))()
    off = 0
    soff = 0
    offsets, support_offsets, shapes = [], [], []
    for d, im in zip(descs, images):
        m, n = int(im["m"]), int(im["n"])
        d.offset = off
        d.m, d.n = m, n
        d.lam = float(im["lam"])
        d.tv_kind = _lib.KINDS[im.get("kind", "1i")]
        d.alpha = float(im.get("alpha", 0.5))
        d.iters = int(im.get("iters", 100))
        if im.get("has_support"):
            d.support_offset = soff
            support_offsets.append(soff)
            soff += m * n
        else:
            d.support_offset = -1
            support_offsets.append(-1)
        offsets.append(off)
        shapes.append((m, n))
        off += m * n
    return descs, offsets, support_offsets, shapes, off, soff


def _tunings(arr, count):
    return [dict(fuse=arr[i].fuse, tile=(arr[i].tile_waves, arr[i].tile_rows), ms=arr[i].ms) for i in range(count)]


_MAX_CANDIDATES = 64


def autotune(b, lam, kind="1i", alpha=0.5, constraint="modulus", support=None, iters=100, method="fgp", reps=3,
             out=None, workspace=None):
    """Times every candidate (tile shape, fuse) for this problem with
    ctv_autotune and records the fastest for the process; later automatic
    calls of ``denoise`` (and ``tiling``, and the prox of ``phase_retrieval``)
    with the same kind, constraint, method, batch, size and iters use it.
    Returns {"best": {...}, "candidates": [...]}; ``out`` (if given) holds the
    solution afterwards."""
    _require_cuda(b, "b", torch.complex64)
    bb = b.unsqueeze(0) if b.dim() == 2 else b
    B, m, n = bb.shape
    dev = bb.device
    p = make_params(kind, alpha, constraint, iters, 0, method=method)
    if support is not None:
        _require_cuda(support, "support", torch.uint8)
    x = _out_like(out, b)
    ws_bytes, _ = workspace_size(m, n, B, kind, alpha, constraint, iters, 0, 0, method)
    ws = workspace if workspace is not None else torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    res = (_lib.Tuning * _MAX_CANDIDATES)()
    cnt = ctypes.c_int32()
    best = _lib.Tuning()
    call("ctv_autotune", ctypes.byref(p), B, m, n, _ptr(bb), _lams(lam, B), _ptr(support), _ptr(x), _ptr(ws),
         ws.numel(), int(reps), res, _MAX_CANDIDATES, ctypes.byref(cnt), ctypes.byref(best), _stream(dev))
    return {"best": _tunings([best], 1)[0], "candidates": _tunings(res, min(cnt.value, _MAX_CANDIDATES))}


def autotune_batched(images, b_packed, support_packed=None, constraint="modulus", method="fgp", reps=3, out=None):
    """ctv_batched_autotune for a ragged batch (``images`` as for BatchedPlan,
    ``b_packed`` packed in the same order): a BatchedPlan of these images
    created afterwards with fuse 0 uses the fastest configuration."""
    _require_cuda(b_packed, "b_packed", torch.complex64)
    dev = b_packed.device
    descs = _image_descs(images)[0]
    common = make_params("1i", 0.5, constraint, 0, 0, method=method)
    x = out if out is not None else torch.empty_like(b_packed)
    sizing = BatchedPlan(images, constraint, fuse=8, method=method)  # workspace size only
    ws_bytes = sizing.ws_bytes
    sizing.close()
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
    res = (_lib.Tuning * _MAX_CANDIDATES)()
    cnt = ctypes.c_int32()
    best = _lib.Tuning()
    call("ctv_batched_autotune", descs, len(images), ctypes.byref(common), _ptr(b_packed), _ptr(support_packed),
         _ptr(x), _ptr(ws), ws.numel(), int(reps), res, _MAX_CANDIDATES, ctypes.byref(cnt), ctypes.byref(best),
         _stream(dev))
    return {"best": _tunings([best], 1)[0], "candidates": _tunings(res, min(cnt.value, _MAX_CANDIDATES))}


def tuned(m, n, batch=1, kind="1i", alpha=0.5, constraint="modulus", iters=100, method="fgp"):
    """The recorded configuration {"fuse", "tile"} for this plain problem on
    the current device, or None."""
    p = make_params(kind, alpha, constraint, iters, 0, method=method)
    found = ctypes.c_int32()
    e = _lib.Tuning()
    call("ctv_tune_lookup", ctypes.byref(p), batch, m, n, ctypes.byref(found), ctypes.byref(e))
    return dict(fuse=e.fuse, tile=(e.tile_waves, e.tile_rows)) if found.value else None


def batched_tuned(images, constraint="modulus", method="fgp"):
    """The recorded configuration {"fuse", "tile"} for a batched plan of these
    images on the current device, or None."""
    descs = _image_descs(images)[0]
    common = make_params("1i", 0.5, constraint, 0, 0, method=method)
    found = ctypes.c_int32()
    e = _lib.Tuning()
    call("ctv_batched_tune_lookup", descs, len(images), ctypes.byref(common), ctypes.byref(found), ctypes.byref(e))
    return dict(fuse=e.fuse, tile=(e.tile_waves, e.tile_rows)) if found.value else None


def tune_cache_save(path):
    """Writes the tuning table (one JSON object per line)."""
    call("ctv_tune_cache_save", str(path).encode())


def tune_cache_load(path):
    """Merges a saved tuning table into the process's table."""
    call("ctv_tune_cache_load", str(path).encode())


def tune_cache_clear():
    call("ctv_tune_cache_clear")


def tune_cache_size():
    return int(_lib.lib().ctv_tune_cache_size())


class BatchedPlan:
    """Ragged batch of images denoised in one HIP-graph launch.

    images: list of dicts with keys m, n, lam, kind ('1i'..'2a'), alpha,
    iters and optionally has_support. Images are packed back to back in the
    order given; ``offsets`` gives each image's first pixel.
    """

    def __init__(self, images, constraint="modulus", fuse=0, method="fgp", tile=(0, 0)):
        descs, self.offsets, self.support_offsets, self.shapes, self.total_pixels, self.support_bytes = \
            _image_descs(images)
        common = make_params("1i", 0.5, constraint, 0, fuse, tile, method=method)
        h = ctypes.c_void_p()
        call("ctv_batched_plan_create", descs, len(images), ctypes.byref(common), ctypes.byref(h))
        self._h = h
        ws = ctypes.c_size_t()
        call("ctv_batched_workspace_size", self._h, ctypes.byref(ws))
        self.ws_bytes = ws.value
        self._ws = None

    @property
    def tiling(self):
        """(iterations fused per launch, tile_waves, tile_rows) of the plan."""
        f, w, r = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        call("ctv_batched_plan_tiling", self._h, ctypes.byref(f), ctypes.byref(w), ctypes.byref(r))
        return f.value, w.value, r.value

    def pack(self, imgs, device="cuda"):
        flat = torch.empty(self.total_pixels, dtype=torch.complex64, device=device)
        for o, (m, n), im in zip(self.offsets, self.shapes, imgs):
            flat[o:o + m * n] = torch.as_tensor(im).reshape(-1).to(device=device, dtype=torch.complex64)
        return flat

    def pack_support(self, masks, device="cuda"):
        """Packs the masks of the images declared with has_support (in order)."""
        flat = torch.zeros(max(self.support_bytes, 1), dtype=torch.uint8, device=device)
        it = iter(masks)
        for so, (m, n) in zip(self.support_offsets, self.shapes):
            if so >= 0:
                flat[so:so + m * n] = torch.as_tensor(next(it)).reshape(-1).to(device=device, dtype=torch.uint8)
        return flat

    def unpack(self, flat):
        return [flat[o:o + m * n].reshape(m, n) for o, (m, n) in zip(self.offsets, self.shapes)]

    def run(self, b_packed, support_packed=None, out=None):
        _require_cuda(b_packed, "b_packed", torch.complex64)
        dev = b_packed.device
        x = out if out is not None else torch.empty_like(b_packed)
        if self._ws is None or self._ws.device != dev:
            self._ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=dev)
        call("ctv_denoise_batched", self._h, _ptr(b_packed), _ptr(support_packed), _ptr(x), _ptr(self._ws),
             self._ws.numel(), _stream(dev))
        return x

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            call("ctv_batched_plan_destroy", self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _pr_params(distances, wavelength, pixel, tau, gamma, outer, inner_iters, kind, alpha, constraint,
               init_backprop, accelerate, fuse, inner_method="fgp", line_search=False, shrink=0.5, max_trials=20,
               warm_start=False):
    dist = (ctypes.c_double * len(distances))(*[float(d) for d in distances])
    p = _lib.PrParams(ctypes.sizeof(_lib.PrParams), len(distances), dist, float(wavelength), float(pixel),
                      float(tau), float(gamma), int(outer), make_params(kind, alpha, constraint, inner_iters, fuse,
                                                                     method=inner_method),
                      int(init_backprop), int(accelerate), int(bool(line_search)), float(shrink), int(max_trials),
                      int(bool(warm_start)))
    return p, dist


def _pr_ws(p, m, n, dev):
    ws = ctypes.c_size_t()
    call("pr_workspace_size", ctypes.byref(p), m, n, ctypes.byref(ws))
    return torch.empty(max(ws.value, 1), dtype=torch.uint8, device=dev)


def phase_retrieval(y, distances, wavelength, pixel, tau=0.01, gamma=0.0, outer=100, inner=20, kind="1i",
                    alpha=0.5, constraint="modulus", x0=None, accelerate=True, fuse=0, loss=False,
                    inner_method="fgp", line_search=False, shrink=0.5, max_trials=20, warm_start=False,
                    steps=False):
    """Algorithm 1 with the FGP prox (inner_method "gp": the Eq. 21 prox);
    y: float32 CUDA [D, m, n] intensities. line_search: backtracking step
    (factor `shrink`, at most `max_trials` prox evaluations per outer
    iteration, starting from `gamma`); warm_start: each prox starts from the
    previous one's last dual iterate. Returns x, then the data-term trace
    (loss=True) and the step used per outer iteration (steps=True)."""
    _require_cuda(y, "y", torch.float32)
    D, m, n = y.shape
    dev = y.device
    p, _keep = _pr_params(distances, wavelength, pixel, tau, gamma, outer, inner, kind, alpha, constraint,
                          x0 is None, accelerate, fuse, inner_method, line_search, shrink, max_trials, warm_start)
    x = torch.empty((m, n), dtype=torch.complex64, device=dev) if x0 is None else x0.clone()
    lt = torch.empty(max(outer, 1), dtype=torch.float32, device=dev) if loss else None
    gt = torch.empty(max(outer, 1), dtype=torch.float32, device=dev) if steps else None
    ws = _pr_ws(p, m, n, dev)
    call("pr_prox_grad", ctypes.byref(p), m, n, _ptr(y), _ptr(x), _ptr(lt), _ptr(gt), _ptr(ws), ws.numel(),
         _stream(dev))
    res = [x]
    if loss:
        res.append(lt[:outer])
    if steps:
        res.append(gt[:outer])
    return res[0] if len(res) == 1 else tuple(res)


def phase_retrieval_ip(y, distances, wavelength, pixel, iters=100, constraint="modulus", x0=None, loss=False):
    """The iterative projection comparison method of Section VI-A (pr_ip): per
    iteration, the measured-modulus projection of each distance in turn, each
    followed by P_C (constraint "modulus": Eq. 25; "none": C = C^{m x n}).
    y: float32 CUDA [D, m, n]. Starts from the back-propagated field unless x0
    is given. Returns x (and the data-term trace F(x_k) with loss=True)."""
    _require_cuda(y, "y", torch.float32)
    D, m, n = y.shape
    dev = y.device
    p, _keep = _pr_params(distances, wavelength, pixel, 0.0, 0.0, iters, 0, "1i", 0.5, constraint, x0 is None, 0, 0)
    x = torch.empty((m, n), dtype=torch.complex64, device=dev) if x0 is None else x0.clone()
    lt = torch.empty(max(iters, 1), dtype=torch.float32, device=dev) if loss else None
    ws = _pr_ws(p, m, n, dev)
    call("pr_ip", ctypes.byref(p), m, n, _ptr(y), _ptr(x), _ptr(lt), _ptr(ws), ws.numel(), _stream(dev))
    return (x, lt[:iters]) if loss else x


def pr_forward(x, distances, wavelength, pixel):
    _require_cuda(x, "x", torch.complex64)
    m, n = x.shape
    p, _keep = _pr_params(distances, wavelength, pixel, 0, 1, 0, 0, "1i", 0.5, "modulus", 0, 1, 0)
    out = torch.empty((len(distances), m, n), dtype=torch.complex64, device=x.device)
    ws = _pr_ws(p, m, n, x.device)
    call("pr_forward", ctypes.byref(p), m, n, _ptr(x), _ptr(out), _ptr(ws), ws.numel(), _stream(x.device))
    return out


def pr_gradient(x, y, distances, wavelength, pixel):
    _require_cuda(x, "x", torch.complex64)
    _require_cuda(y, "y", torch.float32)
    m, n = x.shape
    p, _keep = _pr_params(distances, wavelength, pixel, 0, 1, 0, 0, "1i", 0.5, "modulus", 0, 1, 0)
    g = torch.empty_like(x)
    lv = torch.empty(1, dtype=torch.float32, device=x.device)
    ws = _pr_ws(p, m, n, x.device)
    call("pr_gradient", ctypes.byref(p), m, n, _ptr(y), _ptr(x), _ptr(g), _ptr(lv), _ptr(ws), ws.numel(),
         _stream(x.device))
    return g, lv


def fft2(x, inverse=False):
    _require_cuda(x, "x", torch.complex64)
    squeeze = x.dim() == 2
    xx = x.unsqueeze(0) if squeeze else x
    B, m, n = xx.shape
    out = torch.empty_like(xx)
    wsb = ctypes.c_size_t()
    call("ctv_fft2_workspace_size", B, m, n, ctypes.byref(wsb))
    ws = torch.empty(max(wsb.value, 1), dtype=torch.uint8, device=x.device)
    call("ctv_fft2", B, m, n, _ptr(xx), _ptr(out), int(bool(inverse)), _ptr(ws), ws.numel(), _stream(x.device))
    return out[0] if squeeze else out
