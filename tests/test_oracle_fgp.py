"""Pins for the oracle FGP (Algorithm 2 + Eq. 18): special cases, the real
reduction against an independently written real solver, equivariances at equal
iteration count, the duality gap, closed forms and a brute-force certificate."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import pdhg, real_fgp, tv


def rand_img(shape, rng, scale=0.8):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * scale


# ----------------------------------------------------------------------------
# special cases
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("kind", tv.KINDS)
def test_lambda_zero_and_K_zero_give_PC(kind, rng):
    b = rand_img((6, 5), rng, 1.2)
    mask = (rng.random((6, 5)) > 0.3).astype(np.uint8)
    for mk in (None, mask):
        pu, pv = tv.P_C(b.real, b.imag, "modulus", mk)
        for x in (tv.fgp(b, 0.0, 30, kind, mask=mk), tv.fgp(b, 0.4, 0, kind, mask=mk)):
            np.testing.assert_array_equal(x, pu + 1j * pv)


@pytest.mark.parametrize("kind", tv.KINDS)
def test_output_in_C_and_mask_exactly_zero(kind, rng):
    b = rand_img((9, 8), rng, 1.5)
    mask = (rng.random((9, 8)) > 0.3).astype(np.uint8)
    x = tv.fgp(b, 0.2, 40, kind, mask=mask)
    assert np.all(np.abs(x) <= 1 + 1e-15)
    assert np.all(x[mask == 0] == 0)


@pytest.mark.parametrize("kind", tv.KINDS)
def test_real_input_matches_independent_real_fgp(kind, rng):
    """Real b: Im x stays exactly 0; type-I equals the real constrained FGP at
    the same lam, type-II at lam*alpha (the dual radius alpha rescales the
    iteration exactly)."""
    b = rng.standard_normal((7, 9)) * 1.3
    alpha = 0.5 if kind[0] == "1" else 0.3
    lam = 0.15
    K = 60
    x = tv.fgp(b + 0j, lam, K, kind, alpha)
    assert np.all(x.imag == 0)
    iso = kind.endswith("i")
    if kind[0] == "1":
        xr, _, _ = real_fgp.real_fgp(b, lam, K, iso=iso)
    else:
        xr, _, _ = real_fgp.real_fgp(b, lam * alpha, K, iso=iso)
        xr2, _, _ = real_fgp.real_fgp(b, lam, K, iso=iso, radius=alpha)
        np.testing.assert_allclose(xr2, xr, atol=1e-13)
    np.testing.assert_allclose(x.real, xr, atol=1e-13)


@pytest.mark.parametrize("kind", tv.KINDS)
def test_resume_equals_continuous(kind, rng):
    b = rand_img((6, 7), rng)
    x_full = tv.fgp(b, 0.2, 25, kind)
    _, st = tv.fgp(b, 0.2, 10, kind, return_state=True)
    x_res = tv.fgp(b, 0.2, 15, kind, state=st)
    np.testing.assert_array_equal(x_res, x_full)


# ----------------------------------------------------------------------------
# equivariances that hold at every iteration count
# ----------------------------------------------------------------------------

def test_equivariances(rng):
    b = rand_img((6, 8), rng)
    mask = (rng.random((6, 8)) > 0.25).astype(np.uint8)
    lam, K = 0.17, 35
    th = np.exp(1j * 0.77)
    for kind in tv.KINDS:
        for mk in (None, mask):
            x = tv.fgp(b, lam, K, kind, mask=mk)
            # conjugation: all kinds
            np.testing.assert_allclose(tv.fgp(np.conj(b), lam, K, kind, mask=mk), np.conj(x), atol=1e-13)
            # transpose (directions swap): all kinds
            mt = None if mk is None else mk.T
            np.testing.assert_allclose(tv.fgp(b.T, lam, K, kind, mask=mt), x.T, atol=1e-13)
            if kind[0] == "1":
                # global phase rotation: type-I only
                np.testing.assert_allclose(tv.fgp(th * b, lam, K, kind, mask=mk), th * x, atol=1e-13)
            if kind.endswith("a"):
                # flips: anisotropic only
                mf = None if mk is None else mk[::-1, :]
                np.testing.assert_allclose(tv.fgp(b[::-1, :], lam, K, kind, mask=mf), x[::-1, :], atol=1e-13)
                mf = None if mk is None else mk[:, ::-1]
                np.testing.assert_allclose(tv.fgp(b[:, ::-1], lam, K, kind, mask=mf), x[:, ::-1], atol=1e-13)
    for kind in ("2i", "2a"):
        # multiplication by i swaps the planes: type-II with alpha = 1/2
        x = tv.fgp(b, lam, K, kind, 0.5)
        np.testing.assert_allclose(tv.fgp(1j * b, lam, K, kind, 0.5), 1j * x, atol=1e-13)


def test_isotropic_is_not_flip_symmetric(rng):
    """Sanity check of the test above: forward-difference isotropic TV pairs
    differences at one corner, so a flip changes the iterates."""
    b = rand_img((6, 8), rng)
    x = tv.fgp(b, 0.3, 30, "1i")
    assert np.abs(tv.fgp(b[::-1, :], 0.3, 30, "1i") - x[::-1, :]).max() > 1e-6


# ----------------------------------------------------------------------------
# duality gap
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("kind", tv.KINDS)
@pytest.mark.parametrize("constraint", tv.CONSTRAINTS)
def test_gap_two_ways_nonnegative_and_decreasing(kind, constraint, rng):
    b = rand_img((8, 8), rng, 1.0)
    mask = (rng.random((8, 8)) > 0.2).astype(np.uint8)
    st = None
    gaps = []
    for _ in range(6):
        _, st = tv.fgp(b, 0.25, 50, kind, 0.4, constraint, mask, state=st, return_state=True)
        g1 = tv.gap_primal_minus_dual(st[0], b, 0.25, kind, 0.4, constraint, mask)
        g2, gmin = tv.gap_groups(st[0], b, 0.25, kind, 0.4, constraint, mask)
        assert abs(g1 - g2) <= 1e-10 * max(1.0, abs(g1))
        assert gmin >= -1e-12
        gaps.append(g2)
    assert gaps[-1] < 0.2 * gaps[0] + 1e-12


# ----------------------------------------------------------------------------
# closed forms and brute force
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("kind", tv.KINDS)
def test_two_pixel_closed_form(kind, rng):
    """A 1x2 (or 2x1) image has one difference. Without a modulus bound the
    minimiser moves each pixel toward the other by min(lam*w, |d|/2) along the
    difference (type-I: complex modulus, w = 1; type-II: per plane, w = alpha
    or 1 - alpha)."""
    alpha = 0.3
    lam = 0.2
    for shape in ((1, 2), (2, 1)):
        b = rand_img(shape, rng, 0.5)
        b1, b2 = b.ravel()
        if kind[0] == "1":
            d = b1 - b2
            s = min(lam, abs(d) / 2)
            x1, x2 = b1 - s * d / abs(d), b2 + s * d / abs(d)
        else:
            parts = []
            for f, w in ((np.real, alpha), (np.imag, 1 - alpha)):
                d = f(b1) - f(b2)
                s = min(lam * w, abs(d) / 2)
                parts.append((f(b1) - s * np.sign(d), f(b2) + s * np.sign(d)))
            x1 = parts[0][0] + 1j * parts[1][0]
            x2 = parts[0][1] + 1j * parts[1][1]
        x = tv.fgp(b, lam, 3000, kind, alpha, "none")
        np.testing.assert_allclose(x.ravel(), [x1, x2], atol=1e-9)


@pytest.mark.parametrize("constraint", tv.CONSTRAINTS)
def test_large_lambda_gives_projected_mean(constraint, rng):
    b = rand_img((8, 8), rng, 0.6) + (0.9 + 0.5j)
    x = tv.fgp(b, 30.0, 4000, "1i", constraint=constraint)
    mu = b.mean()
    if constraint == "modulus":
        mu = mu / max(1.0, abs(mu))
    np.testing.assert_allclose(x, np.full(b.shape, mu), atol=1e-6)
    mask = np.ones((8, 8), np.uint8)
    mask[2, 3] = 0
    x = tv.fgp(b, 30.0, 4000, "1i", constraint=constraint, mask=mask)
    np.testing.assert_allclose(x, 0, atol=1e-6)


@pytest.mark.parametrize("kind", tv.KINDS)
@pytest.mark.parametrize("shape,masked", [((4, 4), False), ((4, 4), True), ((3, 5), False)])
def test_fgp_converges_to_brute_force_minimiser(kind, shape, masked, rng):
    """Long FGP runs reach the minimiser of Eq. (1): the gap certificate of its
    (x, lam*q), evaluated with the dense matrix and groups of ``oracle.pdhg``,
    is ~0, and the independent primal-dual solve agrees within the sum of the
    two certificates' distance bounds."""
    b = rand_img(shape, rng, 0.9)
    mask = None
    if masked:
        mask = np.ones(shape, np.uint8)
        mask[1, 2] = 0
        mask[0, 0] = 0
    lam = 0.3
    x, (q, _, _) = tv.fgp(b, lam, 15000, kind, 0.5, "modulus", mask, return_state=True)
    prob = pdhg.Problem(b, lam, kind, 0.5, "modulus", mask)
    y = pdhg.dual_to_vec(q, lam)
    assert prob.in_dual_set(y)
    cert_f = prob.certificate(pdhg.to_vec(x), y)
    assert -1e-12 <= cert_f <= 1e-11
    xp, yp, cert_p = pdhg.solve(b, lam, kind, 0.5, "modulus", mask, iters=20000)
    assert cert_p >= -1e-12
    bound = np.sqrt(2 * max(cert_p, 0)) + np.sqrt(2 * max(cert_f, 0)) + 1e-12
    assert np.linalg.norm(pdhg.to_vec(xp) - pdhg.to_vec(x)) <= bound


def test_paper_qualitative_regularisation_strength():
    """Section IV-C: at a fixed lambda, type-I smooths more than type-II and
    anisotropic more than isotropic (measured as the TV1i of the output), on a
    synthetic unit-modulus phase image with N(0, (pi/10)^2) phase noise."""
    const = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
    f1 = const["fig1_denoising"]
    rng = np.random.default_rng(7)
    ph = np.angle(synth.piecewise_complex(48, 48, 8, rng))
    b = np.exp(1j * (ph + rng.normal(0, np.pi * f1["phase_noise_std_over_pi"], ph.shape)))
    lam = 0.2
    out = {k: tv.tv(tv.fgp(b, lam, f1["iters"], k, f1["alpha"]), "1i") for k in tv.KINDS}
    assert out["1i"] < out["2i"] and out["1a"] < out["2a"]
    assert out["1a"] < out["1i"] and out["2a"] < out["2i"]


@pytest.mark.parametrize("kind", tv.KINDS)
def test_gradient_projection_variant(kind, rng):
    """Eq. (21): the unaccelerated iteration equals the independent real solver
    with acceleration off, differs from FGP at equal K, and reaches the same
    minimiser (brute-force certificate)."""
    b = rng.standard_normal((6, 7)) * 1.3
    lam, K = 0.15, 40
    x = tv.fgp(b + 0j, lam, K, kind, 0.5, method="gp")
    xr, _, _ = real_fgp.real_fgp(b, lam if kind[0] == "1" else lam * 0.5, K, iso=kind.endswith("i"),
                                 accelerate=False)
    np.testing.assert_allclose(x.real, xr, atol=1e-13)
    bc = rand_img((4, 4), rng, 0.9)
    xg, (q, _, _) = tv.fgp(bc, 0.3, 20000, kind, method="gp", return_state=True)
    prob = pdhg.Problem(bc, 0.3, kind, 0.5)
    assert prob.certificate(pdhg.to_vec(xg), pdhg.dual_to_vec(q, 0.3)) <= 1e-10
    assert np.abs(tv.fgp(bc, 0.3, 15, kind, method="gp") - tv.fgp(bc, 0.3, 15, kind)).max() > 1e-6


@pytest.mark.parametrize("kind", tv.KINDS)
def test_dependence_radius_is_one_pixel_per_iteration(kind, rng):
    """x after K iterations depends on b only within Chebyshev distance K + 1:
    on a corner crop the oracle reproduces the full-image result wherever the
    pixel is at least K + 2 away from the cut edges (the basis of the sampled
    full-size parity checks), and not everywhere (the bound is not vacuous)."""
    b = rand_img((40, 44), rng, 1.2)
    mask = (rng.random((40, 44)) > 0.2).astype(np.uint8)
    K, lam = 6, 0.3
    full = tv.fgp(b, lam, K, kind, 0.4, "modulus", mask)
    for (r0, r1, c0, c1) in ((0, 22, 0, 25), (17, 40, 20, 44)):
        crop = tv.fgp(b[r0:r1, c0:c1], lam, K, kind, 0.4, "modulus", mask[r0:r1, c0:c1])
        m = K + 2
        rs = slice(0 if r0 == 0 else m, (r1 - r0) if r1 == 40 else (r1 - r0) - m)
        cs = slice(0 if c0 == 0 else m, (c1 - c0) if c1 == 44 else (c1 - c0) - m)
        np.testing.assert_allclose(crop[rs, cs], full[r0:r1, c0:c1][rs, cs], atol=1e-13)
        assert np.abs(crop - full[r0:r1, c0:c1]).max() > 1e-8


# ----------------------------------------------------------------------------
# the dual outside the support
# ----------------------------------------------------------------------------

def _dead_pixels(mask):
    """Pixels outside the support whose lower and right neighbours (where they
    exist) are outside it too."""
    m = mask.astype(bool)
    live = m.copy()
    live[:-1, :] |= m[1:, :]
    live[:, :-1] |= m[:, 1:]
    return ~live


@pytest.mark.parametrize("kind", tv.KINDS)
@pytest.mark.parametrize("constraint", ["modulus", "none"])
def test_dual_stays_zero_where_no_support_pixel_reaches_it(kind, constraint, rng):
    """From q_0 = 0 (Algorithm 2, line 1) every dual group at a pixel that is
    outside the support, and whose lower and right neighbours are outside it as
    well, is exactly zero after any number of iterations: y = P_C(w) vanishes
    at all three pixels that enter its difference (Eqs. 5-6), so the gradient
    step adds nothing and P_S(0) = 0. The GPU path skips tiles made only of such
    pixels. The group just above or left of a support pixel does move, so the
    neighbours cannot be dropped from the rule."""
    m, n = 23, 19
    b = rand_img((m, n), rng, 1.3)
    mask = np.zeros((m, n), np.uint8)
    mask[6:15, 4:12] = 1
    mask[m - 1, n - 1] = 1
    mask[0, 17] = 1
    dead = _dead_pixels(mask)
    x, (q, _, _) = tv.fgp(b, 0.15, 37, kind, 0.5, constraint, mask, return_state=True)
    r1, r2, s1, s2 = q
    at = np.zeros((m, n), bool)         # any nonzero component of the group at (j, k)
    at[:-1, :] |= (r1 != 0) | (s1 != 0)
    at[:, :-1] |= (r2 != 0) | (s2 != 0)
    assert not np.any(at & dead)
    assert np.all(x[mask == 0] == 0)
    fringe = ~dead & (mask == 0)
    assert np.any(at & fringe)          # the groups next to the support are not zero
