"""GPU tests of ctv_denoise_backward: the hand-written reverse pass agrees with
the oracle's reverse pass (same incoming gradient) and, on the full 16 x 512^2
batch with checkpoints every 10 iterations, with FP64 central finite
differences (h = 1e-6) of the oracle's forward map to 1e-4."""
import numpy as np
import pytest

import synth
from _parity import elem
from oracle import adjoint as oadj
from oracle import tv

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

TOL = 1e-4


def ctv():
    import paper_2109_05496_amd as m
    return m


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def gpu_vjp(b, lam, K, xbar, kind, alpha=0.5, constraint="modulus", mask=None, ckpt=10, method="fgp"):
    """Always runs a batch (a single image becomes a batch of one)."""
    if b.ndim == 2:
        b, xbar = b[None], xbar[None]
    bt = dev(b.astype(np.complex64))
    lams = lam if isinstance(lam, (list, tuple)) else [lam]
    mk = None if mask is None else dev(mask)
    x, saved = ctv().denoise(bt, lams, kind=kind, alpha=alpha, constraint=constraint, support=mk, iters=K,
                             ckpt_every=ckpt, method=method)
    gb, gl = ctv().denoise_backward(bt, lams, dev(xbar.astype(np.complex64)), saved, kind=kind, alpha=alpha,
                                    constraint=constraint, support=mk, iters=K, ckpt_every=ckpt, method=method)
    torch.cuda.synchronize()
    return x.cpu().numpy(), gb.cpu().numpy(), gl.cpu().numpy()


def case(shape, seed, scale=1.4):
    rng = np.random.default_rng(seed)
    _, b = synth.denoise_case(shape[0], shape[1], 5, 0.15, rng)
    xbar = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
    return (b * scale).astype(np.complex64), xbar


@pytest.mark.parametrize("kind", tv.KINDS)
@pytest.mark.parametrize("constraint", ["modulus", "none"])
@pytest.mark.parametrize("shape,K", [((37, 53), 7), ((1, 40), 20), ((45, 1), 23), ((70, 90), 23)])
def test_backward_matches_oracle_reverse(kind, constraint, shape, K):
    b, xbar = case(shape, 3)
    lam, alpha = 0.07, 0.35
    _, gb, gl = gpu_vjp(b, lam, K, xbar, kind, alpha, constraint)
    _, gbo, glo = oadj.fgp_vjp(b.astype(np.complex128), lam, K, xbar.astype(np.complex128), kind, alpha, constraint)
    print("adjoint", kind, constraint, shape, K, "grad_b rel-L2", rel(gb[0], gbo), "elementwise", elem(gb[0], gbo),
          "grad_lambda rel", abs(gl[0] - glo) / max(1.0, abs(glo)))
    assert rel(gb[0], gbo) <= TOL, (kind, constraint, shape, K, rel(gb[0], gbo))
    assert abs(gl[0] - glo) <= TOL * max(1.0, abs(glo)), (gl[0], glo)


def test_backward_8192_local_cotangent_against_oracle_on_a_crop():
    """Masked 8192^2, type-1i, K = 10 with checkpoints every 5 (1 GiB per dual
    plane; the recomputed r history 5 GiB): a cotangent nonzero only on a
    48 x 48 window inside the support near its bottom-right corner. x there
    depends on b within distance K + 1 only, so grad_b must vanish exactly
    outside a crop with a margin of 2 (K + 2) around the window, and the
    oracle's reverse pass on that crop gives grad_b and grad_lambda (the
    iterates it needs lie at least K + 2 from the crop's cut edges)."""
    c = synth.config2(0, size=8192, n_shapes=40)
    b, mask = c["b"], c["mask"]
    m, n = b.shape
    K, ck, lam = 10, 5, c["lam"]
    rows = np.flatnonzero(mask.any(axis=1))
    cols = np.flatnonzero(mask.any(axis=0))
    W = 48
    r0, c0 = int(rows[-1]) - 100, int(cols[-1]) - 100
    rng = np.random.default_rng(21)
    xbar = np.zeros((m, n), dtype=np.complex64)
    xbar[r0:r0 + W, c0:c0 + W] = (rng.standard_normal((W, W)) + 1j * rng.standard_normal((W, W))).astype(np.complex64)
    _, gb, gl = gpu_vjp(b, lam, K, xbar, "1i", 0.5, "modulus", mask, ckpt=ck)
    M = 2 * (K + 2)
    R0, R1, C0, C1 = max(r0 - M, 0), min(r0 + W + M, m), max(c0 - M, 0), min(c0 + W + M, n)
    outside = np.ones((m, n), dtype=bool)
    outside[R0:R1, C0:C1] = False
    assert not np.any(gb[0][outside]), "grad_b nonzero beyond the cotangent's dependency cone"
    _, gbo, glo = oadj.fgp_vjp(b[R0:R1, C0:C1].astype(np.complex128), lam, K,
                               xbar[R0:R1, C0:C1].astype(np.complex128), "1i", 0.5, "modulus",
                               mask[R0:R1, C0:C1])
    got = gb[0][R0:R1, C0:C1]
    print("adjoint 8192 crop grad_b rel-L2", rel(got, gbo), "elementwise", elem(got, gbo),
          "grad_lambda rel", abs(gl[0] - glo) / max(1.0, abs(glo)))
    assert rel(got, gbo) <= TOL
    assert abs(gl[0] - glo) <= TOL * max(1.0, abs(glo)), (gl[0], glo)


@pytest.mark.parametrize("kind", tv.KINDS)
def test_backward_with_mask(kind):
    rng = np.random.default_rng(9)
    b, xbar = case((60, 75), 4)
    mask = synth.square_mask(60, 75, 0.6, rng)
    _, gb, gl = gpu_vjp(b, 0.09, 25, xbar, kind, mask=mask)
    _, gbo, glo = oadj.fgp_vjp(b.astype(np.complex128), 0.09, 25, xbar.astype(np.complex128), kind, 0.5,
                               "modulus", mask)
    print("adjoint masked", kind, "grad_b rel-L2", rel(gb[0], gbo), "elementwise", elem(gb[0], gbo),
          "grad_lambda rel", abs(gl[0] - glo) / max(1.0, abs(glo)))
    assert rel(gb[0], gbo) <= TOL
    assert np.all(gb[0][mask == 0] == 0)
    assert abs(gl[0] - glo) <= TOL * max(1.0, abs(glo))


def test_backward_batch_lambda_zero_and_K_zero():
    rng = np.random.default_rng(2)
    bs = np.stack([case((33, 41), s)[0] for s in range(3)])
    xb = np.stack([case((33, 41), 10 + s)[1] for s in range(3)])
    lams = [0.05, 0.0, 0.12]
    _, gb, gl = gpu_vjp(bs, lams, 12, xb, "1a", ckpt=5)
    for i in range(3):
        _, gbo, glo = oadj.fgp_vjp(bs[i].astype(np.complex128), lams[i], 12, xb[i].astype(np.complex128), "1a")
        assert rel(gb[i], gbo) <= TOL, i
        assert abs(gl[i] - glo) <= TOL * max(1.0, abs(glo)), i
    assert gl[1] == 0.0
    _, gb0, gl0 = gpu_vjp(bs, lams, 0, xb, "1i", ckpt=5)
    for i in range(3):
        _, gbo, _ = oadj.fgp_vjp(bs[i].astype(np.complex128), lams[i], 0, xb[i].astype(np.complex128), "1i")
        assert rel(gb0[i], gbo) <= 1e-6
    assert np.all(gl0 == 0)


def test_autograd_function_matches_backward():
    b, _ = case((48, 64), 5)
    truth = dev(case((48, 64), 6)[0])
    bt = dev(b).requires_grad_(True)
    lam = torch.tensor(0.06, dtype=torch.float32, requires_grad=True)
    x = ctv().CTVDenoise.apply(bt, lam, "1i", 0.5, "modulus", None, 30, 10)
    loss = ((x - truth).abs() ** 2).sum()
    loss.backward()
    xbar = (2 * (x.detach() - truth)).cpu().numpy()
    _, gbo, glo = oadj.fgp_vjp(b.astype(np.complex128), 0.06, 30, xbar.astype(np.complex128), "1i")
    print("autograd grad_b rel-L2", rel(bt.grad.cpu().numpy(), gbo), "grad_lambda", lam.grad.item(), glo)
    assert rel(bt.grad.cpu().numpy(), gbo) <= TOL
    assert abs(lam.grad.item() - glo) <= TOL * max(1.0, abs(glo))


def test_config4_full_batch_against_finite_differences():
    """16 x 512^2, type-1i, lambda 0.05, K = 50, checkpoints every 10, loss
    ||x - truth||^2: directional derivatives of one image (random direction in b,
    and lambda) match FP64 central differences of the oracle forward."""
    c = synth.config4(0)
    b = c["b"]
    truth = c["truth"]
    bt = dev(b).requires_grad_(True)
    lam = torch.full((16,), c["lam"], dtype=torch.float32, requires_grad=True)
    x = ctv().CTVDenoise.apply(bt, lam, "1i", 0.5, "modulus", None, c["iters"], c["ckpt_every"])
    loss = ((x - dev(truth.astype(np.complex64))).abs() ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    i = 5
    gb = bt.grad[i].cpu().numpy().astype(np.complex128)
    gl = float(lam.grad[i])
    rng = np.random.default_rng(0)
    d = rng.standard_normal(b[i].shape) + 1j * rng.standard_normal(b[i].shape)
    h = 1e-6
    b64 = b[i].astype(np.complex128)

    def f(bb, ll):
        return float(np.sum(np.abs(tv.fgp(bb, ll, c["iters"], "1i") - truth[i]) ** 2))

    fd_b = (f(b64 + h * d, c["lam"]) - f(b64 - h * d, c["lam"])) / (2 * h)
    an_b = float(np.sum(gb.real * d.real + gb.imag * d.imag))
    print("config4 directional derivative: FD", fd_b, "GPU adjoint", an_b, "rel", abs(an_b - fd_b) / abs(fd_b))
    assert abs(an_b - fd_b) <= TOL * abs(fd_b)
    fd_l = (f(b64, c["lam"] + h) - f(b64, c["lam"] - h)) / (2 * h)
    print("config4 d/dlambda: FD", fd_l, "GPU adjoint", gl, "rel", abs(gl - fd_l) / abs(fd_l))
    assert abs(gl - fd_l) <= TOL * abs(fd_l)


@pytest.mark.parametrize("kind", ["1i", "2a"])
def test_backward_gradient_projection_method(kind):
    b, xbar = case((52, 67), 12)
    _, gb, gl = gpu_vjp(b, 0.08, 21, xbar, kind, 0.4, ckpt=6, method="gp")
    _, gbo, glo = oadj.fgp_vjp(b.astype(np.complex128), 0.08, 21, xbar.astype(np.complex128), kind, 0.4,
                               method="gp")
    assert rel(gb[0], gbo) <= TOL
    assert abs(gl[0] - glo) <= TOL * max(1.0, abs(glo))
