"""ctv_denoise_noalloc (the entry point for callers that cannot allocate)
against ctv_denoise on the same inputs, through the C ABI: bitwise equal
results (x and the duality gap), on two calls in a row where the second is
smaller (the shared scratch array keeps the first call's contents), and a
problem above the fixed scratch size is refused before any device work."""
import ctypes

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _lib():
    from paper_2109_05496_amd import _lib
    return _lib


def noalloc(b, lams, kind, support=None, iters=40, gap=False):
    """One ctv_denoise_noalloc call on torch-owned input and output buffers."""
    L = _lib()
    B, m, n = b.shape
    x = torch.empty_like(b)
    g = torch.empty(B, dtype=torch.float64, device=b.device) if gap else None
    p = L.make_params(kind, 0.5, "modulus", iters)
    lam = (ctypes.c_float * B)(*lams)
    stream = ctypes.c_void_p(torch.cuda.current_stream(b.device).cuda_stream)
    ptr = (lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None)
    st = L.lib().ctv_denoise_noalloc(ctypes.byref(p), B, m, n, ptr(b), lam, ptr(support), ptr(x), ptr(g), stream)
    L.check("ctv_denoise_noalloc", st)
    return x, g


def reference(b, lams, kind, support=None, iters=40, gap=False):
    import paper_2109_05496_amd as ctv
    r = ctv.denoise(b, lams, kind=kind, support=support, iters=iters, gap=gap)
    return r if gap else (r, None)


def case(B, m, n, seed):
    rng = np.random.default_rng(seed)
    bs = np.stack([synth.denoise_case(m, n, 8, 0.15, rng)[1] for _ in range(B)])
    mask = synth.square_mask(m, n, 0.6, rng)
    return torch.as_tensor(bs).cuda(), torch.as_tensor(mask).cuda()


def same(a, b):
    return torch.equal(a.contiguous().view(torch.uint8), b.contiguous().view(torch.uint8))


def test_two_calls_in_a_row_second_smaller():
    # first call: the largest problem class the scratch holds (1024 x 1024, with a support and the gap)
    b1, m1 = case(1, 1024, 1024, 1)
    x1, g1 = noalloc(b1, [0.08], "2i", support=m1, iters=30, gap=True)
    r1, rg1 = reference(b1, [0.08], "2i", support=m1, iters=30, gap=True)
    # second call: a smaller batch of a different kind, no support
    b2, _ = case(3, 150, 211, 2)
    x2, g2 = noalloc(b2, [0.05, 0.1, 0.2], "1a", iters=23, gap=True)
    r2, rg2 = reference(b2, [0.05, 0.1, 0.2], "1a", iters=23, gap=True)
    torch.cuda.synchronize()
    assert same(x1, r1) and same(g1, rg1)
    assert same(x2, r2) and same(g2, rg2)
    # and once more at the first size after the smaller call
    x3, _ = noalloc(b1, [0.08], "2i", support=m1, iters=30)
    torch.cuda.synchronize()
    assert same(x3, r1)


def test_too_large_problem_is_refused():
    L = _lib()
    p = L.make_params("1i", 0.5, "modulus", 10)
    lam = (ctypes.c_float * 1)(0.1)
    dummy = ctypes.c_void_p(0x1000)
    st = L.lib().ctv_denoise_noalloc(ctypes.byref(p), 1, 2048, 2048, dummy, lam, None, ctypes.c_void_p(0x2000),
                                     None, None)
    assert st == -2
    assert b"workspace" in L.lib().ctv_last_error()
