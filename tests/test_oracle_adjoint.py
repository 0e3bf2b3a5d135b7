"""Pins for the reverse-mode oracle of the K-step FGP map: central finite
differences (float64, h = 1e-6), an independent torch float64 autograd of a
separately written unrolled forward, and the K = 0 closed form."""
import numpy as np
import pytest

from oracle import adjoint, tv

torch = pytest.importorskip("torch")


def case(rng, m=6, n=7):
    b = (rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))) * 0.7
    truth = (rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))) * 0.5
    mask = (rng.random((m, n)) > 0.2).astype(np.uint8)
    return b, truth, mask


@pytest.mark.parametrize("kind", tv.KINDS)
@pytest.mark.parametrize("constraint", tv.CONSTRAINTS)
def test_manual_reverse_equals_torch_autograd(kind, constraint, rng):
    b, truth, mask = case(rng)
    lam, K, alpha = 0.15, 12, 0.4
    for mk in (None, mask):
        x = tv.fgp(b, lam, K, kind, alpha, constraint, mk)
        x2, bb, lb = adjoint.fgp_vjp(b, lam, K, 2 * (x - truth), kind, alpha, constraint, mk)
        np.testing.assert_allclose(x2, x, atol=1e-14)
        br = torch.tensor(b.real, requires_grad=True)
        bi = torch.tensor(b.imag, requires_grad=True)
        lt = torch.tensor(lam, dtype=torch.float64, requires_grad=True)
        xr, xi = adjoint.torch_fgp(br, bi, lt, K, kind, alpha, constraint, mk)
        np.testing.assert_allclose(xr.detach().numpy() + 1j * xi.detach().numpy(), x, atol=1e-13)
        loss = ((xr - torch.tensor(truth.real)) ** 2 + (xi - torch.tensor(truth.imag)) ** 2).sum()
        loss.backward()
        np.testing.assert_allclose(br.grad.numpy() + 1j * bi.grad.numpy(), bb, atol=1e-10)
        assert abs(lt.grad.item() - lb) <= 1e-10 * max(1.0, abs(lb))


@pytest.mark.parametrize("kind", tv.KINDS)
def test_manual_reverse_matches_finite_differences(kind, rng):
    b, truth, mask = case(rng)
    lam, K, alpha, h = 0.12, 15, 0.5, 1e-6
    x = tv.fgp(b, lam, K, kind, alpha, mask=mask)
    _, bb, lb = adjoint.fgp_vjp(b, lam, K, 2 * (x - truth), kind, alpha, mask=mask)

    def loss(bv, lv):
        return float(np.sum(np.abs(tv.fgp(bv, lv, K, kind, alpha, mask=mask) - truth) ** 2))

    for _ in range(3):
        d = rng.standard_normal(b.shape) + 1j * rng.standard_normal(b.shape)
        fd = (loss(b + h * d, lam) - loss(b - h * d, lam)) / (2 * h)
        an = float(np.sum(bb.real * d.real + bb.imag * d.imag))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
    fd = (loss(b, lam + h) - loss(b, lam - h)) / (2 * h)
    assert abs(fd - lb) <= 1e-6 * max(1.0, abs(lb))


def test_K_zero_closed_form(rng):
    b, truth, mask = case(rng)
    b = b * 2.0                       # many pixels outside the unit disc
    pu, pv = tv.P_C(b.real, b.imag, "modulus", mask)
    xbar = 2 * ((pu + 1j * pv) - truth)
    _, bb, lb = adjoint.fgp_vjp(b, 0.3, 0, xbar, mask=mask)
    # closed form of J_{P_C}^T: identity inside the disc, (I - w w^T/|w|^2)/|w| outside
    a = np.abs(b)
    w_hat = b / a
    radial = np.real(np.conj(w_hat) * xbar)
    expect = np.where(a > 1, (xbar - radial * w_hat) / a, xbar) * mask
    np.testing.assert_allclose(bb, expect, atol=1e-14)
    assert lb == 0.0
