"""Pins for the phase-retrieval oracle: the FFT convention against a naive DFT,
the angular-spectrum transfer function's closed-form properties, the data-term
gradient against finite differences and its closed-form special cases, and the
qualitative behaviour of Algorithm 1."""
import math

import numpy as np
import pytest

import synth
from oracle import pr, tv


def naive_dft2(x, sign):
    m, n = x.shape
    Fm = np.exp(sign * 2j * np.pi * np.outer(np.arange(m), np.arange(m)) / m)
    Fn = np.exp(sign * 2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n)
    return Fm @ x @ Fn.T


@pytest.mark.parametrize("shape", [(8, 8), (16, 4), (5, 12)])
def test_fft_convention_matches_naive_dft(shape, rng):
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    np.testing.assert_allclose(np.fft.fft2(x), naive_dft2(x, -1), atol=1e-10)
    np.testing.assert_allclose(np.fft.ifft2(x), naive_dft2(x, +1) / x.size, atol=1e-12)


def test_transfer_function_properties():
    m, n, lam_s, px = 32, 24, 532e-9, 4e-6
    H1 = pr.transfer(m, n, 1.0e-3, lam_s, px)
    H2 = pr.transfer(m, n, 1.5e-3, lam_s, px)
    H12 = pr.transfer(m, n, 2.5e-3, lam_s, px)
    np.testing.assert_allclose(np.abs(H1), 1.0, atol=1e-14)        # all propagating here
    np.testing.assert_allclose(H1 * H2, H12, atol=1e-9)
    np.testing.assert_allclose(pr.transfer(m, n, 0.0, lam_s, px), 1.0, atol=0)
    np.testing.assert_allclose(pr.transfer(m, n, -1.0e-3, lam_s, px), np.conj(H1), atol=1e-12)
    # DC term: phase 2 pi d / lambda exactly
    assert abs(H1[0, 0] - np.exp(2j * np.pi * 1.0e-3 / lam_s)) < 1e-9
    # evanescent band is zero when the grid's highest frequency exceeds 1/lambda
    He = pr.transfer(16, 16, 1e-3, 1.5e-6, 1e-6)
    fx = np.fft.fftfreq(16, 1e-6)
    ev = (1.5e-6 * fx[None, :]) ** 2 + (1.5e-6 * fx[:, None]) ** 2 >= 1
    assert ev.any() and np.all(He[ev] == 0) and np.allclose(np.abs(He[~ev]), 1)


def test_propagator_unitary_and_adjoint(rng):
    m, n = 32, 32
    H = pr.transfer(m, n, 2e-3, 532e-9, 4e-6)
    x = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    z = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    assert abs(np.linalg.norm(pr.A(x, H)) - np.linalg.norm(x)) < 1e-10
    assert abs(np.vdot(z, pr.A(x, H)) - np.vdot(pr.AH(z, H), x)) < 1e-9
    np.testing.assert_allclose(pr.AH(pr.A(x, H), H), x, atol=1e-12)
    Hm = pr.transfer(m, n, -2e-3, 532e-9, 4e-6)
    np.testing.assert_allclose(pr.A(z, Hm), pr.AH(z, H), atol=1e-12)


def small_problem(rng, m=32, D=2):
    truth = synth.config5_object(seed=3, size=m, n_shapes=6, sigma_px=1.5)
    dists = (1.0e-3, 2.0e-3)[:D]
    Hs = [pr.transfer(m, m, d, 532e-9, 4e-6) for d in dists]
    sy = [np.abs(pr.A(truth, H)) for H in Hs]
    return truth, Hs, sy


def test_grad_matches_finite_differences(rng):
    truth, Hs, sy = small_problem(rng)
    x = truth * np.exp(0.3j) + 0.05 * (rng.standard_normal(truth.shape) + 1j * rng.standard_normal(truth.shape))
    g = pr.grad_F(x, sy, Hs)
    h = 1e-6
    for _ in range(3):
        d = rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape)
        fd = (pr.data_term(x + h * d, sy, Hs) - pr.data_term(x - h * d, sy, Hs)) / (2 * h)
        an = float(np.sum(g.real * d.real + g.imag * d.imag))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))


def test_grad_closed_form_cases(rng):
    truth, Hs, sy = small_problem(rng)
    # noise-free data: the truth is a stationary point
    assert np.abs(pr.grad_F(truth, sy, Hs)).max() < 1e-12
    # global phase: grad(e^{i th} x) = e^{i th} grad(x)
    x = truth + 0.1
    th = np.exp(1.1j)
    np.testing.assert_allclose(pr.grad_F(th * x, sy, Hs), th * pr.grad_F(x, sy, Hs), atol=1e-12)
    # one distance, unit step: x - grad F(x) = A^H[ sqrt(y) A x / |A x| ] (magnitude replacement)
    H, s = Hs[0], sy[0]
    Ax = pr.A(x, H)
    mr = pr.AH(s * Ax / np.abs(Ax), H)
    np.testing.assert_allclose(x - pr.grad_F(x, [s], [H]), mr, atol=1e-12)


def test_zero_field_uses_unit_phasor():
    H = pr.transfer(8, 8, 1e-3, 532e-9, 4e-6)
    s = np.ones((8, 8))
    g = pr.grad_F(np.zeros((8, 8), complex), [s], [H])
    np.testing.assert_allclose(g, pr.AH(-np.ones((8, 8)), H), atol=1e-14)


def test_fista_reduces_loss_and_phase_error(rng):
    truth, Hs, sy = small_problem(rng, m=32, D=2)
    y = np.stack([s ** 2 for s in sy])
    x0 = pr.backprop(sy, Hs)
    e0 = pr.phase_rmse(x0, truth)
    x, loss = pr.fista(y, (1.0e-3, 2.0e-3), 532e-9, 4e-6, outer=30, inner=10, tau=0.002, gamma=0.5)
    assert loss[-1] < 0.2 * loss[0]
    assert pr.phase_rmse(x, truth) < e0
    assert np.all(np.abs(x) <= 1 + 1e-12)
    # ISTA (no momentum) is slower than FISTA on the same problem (Fig. 5's observation)
    _, loss_ista = pr.fista(y, (1.0e-3, 2.0e-3), 532e-9, 4e-6, outer=30, inner=10, tau=0.002, gamma=0.5,
                            accelerate=False)
    assert loss[-1] < loss_ista[-1]


def test_phase_rmse_ignores_global_phase(rng):
    truth = synth.config5_object(seed=1, size=16, n_shapes=3, sigma_px=1.0)
    assert pr.phase_rmse(truth * np.exp(2.2j), truth) < 1e-12


def test_line_search_accepts_the_first_step_that_passes_the_model(rng):
    """Backtracking: the accepted step satisfies the quadratic upper model at
    z_1 = x_0 and the step before it (gamma / shrink) did not; steps never grow;
    a small enough start step is accepted at once and reproduces the fixed-step
    iteration exactly."""
    truth, Hs, sy = small_problem(rng, m=32, D=2)
    y = np.stack([s ** 2 for s in sy])
    dists, wl, px = (1.0e-3, 2.0e-3), 532e-9, 4e-6
    kw = dict(outer=5, inner=8, tau=0.002)
    x, loss, info = pr.fista(y, dists, wl, px, gamma=8.0, line_search=True, shrink=0.5, return_info=True, **kw)
    g_steps, trials = info["gamma"], info["trials"]
    assert trials[0] > 1 and np.all(np.diff(g_steps) <= 0)
    x0 = pr.backprop(sy, Hs)
    g = pr.grad_F(x0, sy, Hs)
    F0 = pr.data_term(x0, sy, Hs)

    def passes(gam):
        xc = tv.fgp(x0 - gam * g, 0.002 * gam, 8, "1i")
        d = xc - x0
        model = F0 + np.sum(g.real * d.real + g.imag * d.imag) + np.sum(np.abs(d) ** 2) / (2 * gam)
        return pr.data_term(xc, sy, Hs) <= model

    assert passes(g_steps[0]) and not passes(g_steps[0] / 0.5)
    assert np.isclose(loss[0], F0)
    xs, ls, info_s = pr.fista(y, dists, wl, px, gamma=g_steps[-1], line_search=True, return_info=True, **kw)
    xf, lf = pr.fista(y, dists, wl, px, gamma=g_steps[-1], **kw)
    if np.all(info_s["trials"] == 1):
        np.testing.assert_array_equal(xs, xf)
        np.testing.assert_array_equal(ls, lf)


def test_warm_started_prox_reaches_the_same_minimiser(rng):
    """A warm dual start changes the iterates of a short prox but not its
    limit: with many inner iterations warm and cold starts agree; the first
    outer iteration has no previous dual, so it is identical either way."""
    truth, Hs, sy = small_problem(rng, m=16, D=2)
    y = np.stack([s ** 2 for s in sy])
    dists, wl, px = (1.0e-3, 2.0e-3), 532e-9, 4e-6
    x1c, _ = pr.fista(y, dists, wl, px, outer=1, inner=5, tau=0.01, gamma=0.5)
    x1w, _ = pr.fista(y, dists, wl, px, outer=1, inner=5, tau=0.01, gamma=0.5, warm_start=True)
    np.testing.assert_array_equal(x1c, x1w)
    xs_c, _ = pr.fista(y, dists, wl, px, outer=3, inner=4, tau=0.01, gamma=0.5)
    xs_w, _ = pr.fista(y, dists, wl, px, outer=3, inner=4, tau=0.01, gamma=0.5, warm_start=True)
    assert np.abs(xs_c - xs_w).max() > 1e-8
    xl_c, _ = pr.fista(y, dists, wl, px, outer=3, inner=3000, tau=0.01, gamma=0.5)
    xl_w, _ = pr.fista(y, dists, wl, px, outer=3, inner=3000, tau=0.01, gamma=0.5, warm_start=True)
    np.testing.assert_allclose(xl_w, xl_c, atol=1e-6)


# ---------------------------------------------------------------------------
# Algorithm 1 in closed form. With no measurements (y = 0) the data term of
# Eq. (24) is F(x) = (D/2)||x||^2 on a grid without evanescent frequencies
# (each A_d is unitary), so grad F(x) = D x (Eq. 27 with sqrt(y) = 0). With
# tau = 0 the prox of Eq. (15) is P_C alone (lambda = 0), the identity for
# C = C^{m x n}. Every iterate is then a real multiple of x_0, and the
# multiples obey a scalar recurrence that follows Algorithm 1 step by step:
#   x_k = prox(z_k - gamma D z_k),  t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2,
#   z_{k+1} = x_k + ((t_k - 1) / t_{k+1}) (x_k - x_{k-1}),  z_1 = x_0,  t_1 = 1.
# A momentum index shifted by one, the gradient taken at x_k instead of z_k,
# or z reset to x_k each change the multiples from k = 2 or 3 on.
# ---------------------------------------------------------------------------
_WL, _PX = 532e-9, 4e-6


def _scalar_fista(K, contraction, accelerate=True, clip=None):
    """Multiples (c_z[1..K], c_x[0..K]) of x_0 for the reduced problem:
    x_k = P(contraction * z_k), P = identity or the modulus clip of a
    constant image of modulus `clip` (|.| <= 1 after scaling)."""
    t = 1.0
    cx = [1.0]
    cz = [1.0]
    for k in range(1, K + 1):
        v = contraction * cz[-1]
        if clip is not None:
            v = v / max(1.0, abs(v) * clip)
        cx.append(v)
        t_next = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
        beta = (t - 1.0) / t_next if accelerate else 0.0
        cz.append(cx[k] + beta * (cx[k] - cx[k - 1]))
        t = t_next
    return np.array(cz[:K]), np.array(cx)


def _no_measurement_problem(rng, m=8, n=12, D=1):
    dists = (1.0e-3, 2.5e-3, 1.5e-3)[:D]
    y = np.zeros((D, m, n))
    x0 = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    return y, dists, x0


def test_momentum_sequence_first_values():
    """t_2 = (1 + sqrt 5)/2 (the golden ratio), t_3 = (1 + sqrt(1 + 4 t_2^2))/2 =
    (1 + sqrt(7 + 2 sqrt 5))/2, and t_k >= (k + 1)/2 (Beck and Teboulle's bound);
    at gamma D = 1/2 the multiples are c_x = 1, 1/2, 1/4, (1/8)(1 - beta_2)...
    with beta_2 = (t_2 - 1)/t_3."""
    t2 = (1 + math.sqrt(5)) / 2
    t3 = (1 + math.sqrt(7 + 2 * math.sqrt(5))) / 2
    cz, cx = _scalar_fista(3, 0.5)
    np.testing.assert_allclose(cx[:3], [1.0, 0.5, 0.25], rtol=0, atol=0)
    np.testing.assert_allclose(cz[2], 0.25 - 0.25 * (t2 - 1) / t3, rtol=1e-15)
    np.testing.assert_allclose(cx[3], 0.125 * (1 - (t2 - 1) / t3), rtol=1e-15)
    t = 1.0
    for k in range(1, 200):
        assert t >= (k + 1) / 2 - 1e-12
        t = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0


@pytest.mark.parametrize("D,gamma", [(1, 0.5), (2, 0.25), (3, 0.3)])
def test_fista_iterates_follow_the_scalar_recurrence(rng, D, gamma):
    """Every z_k (through F(z_k) = (D/2) c_z[k]^2 ||x_0||^2, the returned loss
    trace) and the final x_K = c_x[K] x_0 match the recurrence, for one and for
    several distances (the gradient is summed over d)."""
    K = 12
    y, dists, x0 = _no_measurement_problem(rng, D=D)
    x, loss = pr.fista(y, dists, _WL, _PX, outer=K, inner=5, tau=0.0, gamma=gamma,
                       constraint="none", x0=x0)
    cz, cx = _scalar_fista(K, 1.0 - gamma * D)
    nx0 = float(np.sum(np.abs(x0) ** 2))
    np.testing.assert_allclose(loss, 0.5 * D * cz ** 2 * nx0, rtol=1e-11)
    np.testing.assert_allclose(x, cx[K] * x0, rtol=0, atol=1e-12 * np.abs(x0).max())
    # the momentum matters: the same problem without it is the geometric sequence
    xi, li = pr.fista(y, dists, _WL, _PX, outer=K, inner=5, tau=0.0, gamma=gamma,
                      constraint="none", x0=x0, accelerate=False)
    np.testing.assert_allclose(xi, (1.0 - gamma * D) ** K * x0, rtol=0, atol=1e-13 * np.abs(x0).max())
    assert abs(cx[K] - (1.0 - gamma * D) ** K) > 1e-3 * abs(cx[K])


def test_fista_recurrence_with_the_modulus_projection():
    """With C = {|x| <= 1} the prox is the pixelwise projection of Eq. 26. For a
    constant image x_0 = 4 e^{i 0.7} every iterate stays constant, the first prox
    clips (|x_0|/2 = 2 > 1) and later ones do not; the recurrence with the clip
    reproduces all of them (the prox acts after the gradient step, not before)."""
    K = 8
    m, n = 6, 5
    x0 = np.full((m, n), 4.0 * np.exp(0.7j))
    y = np.zeros((1, m, n))
    x, loss = pr.fista(y, (1.0e-3,), _WL, _PX, outer=K, inner=3, tau=0.0, gamma=0.5,
                       constraint="modulus", x0=x0)
    cz, cx = _scalar_fista(K, 0.5, clip=4.0)
    assert cx[1] == 0.25  # 4 * 0.25 = 1: the first prox lands on the circle
    np.testing.assert_allclose(loss, 0.5 * cz ** 2 * 16.0 * m * n, rtol=1e-11)
    np.testing.assert_allclose(x, cx[K] * x0, rtol=0, atol=1e-12)


def test_line_search_steps_in_closed_form(rng):
    """Backtracking on F = (1/2)||x||^2 (one distance, identity prox): the
    quadratic model holds at x = (1 - gamma) z exactly when gamma <= 1
    ((1 - gamma)^2 <= 1 - gamma). Starting from gamma = 3 with shrink 1/2, the
    steps 3 and 1.5 are rejected and 0.75 is accepted on the third trial; later
    iterations keep 0.75 and accept at once, so the iterates follow the
    recurrence with contraction 1/4."""
    K = 6
    y, dists, x0 = _no_measurement_problem(rng, D=1)
    x, loss, info = pr.fista(y, dists, _WL, _PX, outer=K, inner=4, tau=0.0, gamma=3.0,
                             constraint="none", x0=x0, line_search=True, shrink=0.5, return_info=True)
    np.testing.assert_array_equal(info["trials"], [3] + [1] * (K - 1))
    np.testing.assert_array_equal(info["gamma"], [0.75] * K)
    cz, cx = _scalar_fista(K, 0.25)
    np.testing.assert_allclose(loss, 0.5 * cz ** 2 * float(np.sum(np.abs(x0) ** 2)), rtol=1e-11)
    np.testing.assert_allclose(x, cx[K] * x0, rtol=0, atol=1e-12 * np.abs(x0).max())


# ---------------------------------------------------------------------------
# Iterative projection (IP) baseline, Section VI-A.
# ---------------------------------------------------------------------------
def _ip_problem(m=32, D=2, seed=3, noise=False):
    truth = synth.config5_object(seed=seed, size=m, n_shapes=6, sigma_px=1.5)   # |truth| <= 1
    dists = (1.0e-3, 2.0e-3, 1.5e-3)[:D]
    Hs = [pr.transfer(m, m, d, _WL, _PX) for d in dists]
    inten = [np.abs(pr.A(truth, H)) ** 2 for H in Hs]
    if noise:
        rng = np.random.default_rng(seed)
        inten = [synth.poisson_measure(I, 1000.0, rng).astype(np.float64) for I in inten]
    return truth, dists, Hs, np.stack(inten)


def test_ip_noise_free_truth_is_a_fixed_point():
    """With noise-free data and |x_true| <= 1, the truth lies in every
    measured-modulus set and in C, so every projection leaves it in place."""
    truth, dists, Hs, y = _ip_problem(D=3)
    x, loss = pr.ip(y, dists, _WL, _PX, 3, x0=truth)
    np.testing.assert_allclose(x, truth, rtol=0, atol=1e-12)
    assert np.all(loss < 1e-20)


def test_ip_projections_are_idempotent_and_land_in_their_sets(rng):
    truth, dists, Hs, y = _ip_problem(D=1, noise=True)
    sy = np.sqrt(y[0])
    x = truth * np.exp(0.4j) + 0.2 * (rng.standard_normal(truth.shape) + 1j * rng.standard_normal(truth.shape))
    u = pr.project_modulus(x, sy, Hs[0])
    np.testing.assert_allclose(np.abs(pr.A(u, Hs[0])), sy, atol=1e-12)           # in the modulus set
    np.testing.assert_allclose(pr.project_modulus(u, sy, Hs[0]), u, atol=1e-12)   # idempotent
    # the nearest point: no other point of the set among random phase changes is closer
    d0 = np.linalg.norm(u - x)
    for _ in range(5):
        v = pr.AH(sy * np.exp(1j * rng.uniform(-np.pi, np.pi, sy.shape)), Hs[0])
        assert np.linalg.norm(v - x) >= d0 - 1e-12


def test_ip_error_never_increases_with_one_distance():
    """Alternating projections between the modulus set M and the convex set C:
    dist(x_{k+1}, M) <= ||x_{k+1} - P_M x_k|| <= ||x_k - P_M x_k|| = dist(x_k, M),
    and F(x) = dist(x, M)^2 / 2 for a unitary A."""
    truth, dists, Hs, y = _ip_problem(D=1, noise=True)
    # (the back-propagated start already has the measured modulus with one
    # distance, so start elsewhere: a rotated, scaled, noisy copy of the truth)
    rng = np.random.default_rng(4)
    x0 = 1.3 * truth * np.exp(0.7j) + 0.3 * (rng.standard_normal(truth.shape) + 1j * rng.standard_normal(truth.shape))
    _, loss = pr.ip(y, dists, _WL, _PX, 25, x0=x0)
    assert np.all(np.diff(loss) <= 1e-12 * loss[:-1])
    assert loss[-1] < 0.5 * loss[0]


def test_ip_one_distance_equals_a_prox_gradient_step_with_projection_prox():
    """With one distance, x - grad F(x) is the magnitude replacement (Eq. 27),
    so one IP iteration is the proximal gradient step of Eq. (14) with gamma = 1
    and tau = 0 (the prox is P_C alone)."""
    truth, dists, Hs, y = _ip_problem(D=1, noise=True)
    rng = np.random.default_rng(5)
    x0 = 1.3 * truth * np.exp(0.7j) + 0.3 * (rng.standard_normal(truth.shape) + 1j * rng.standard_normal(truth.shape))
    for constraint in ("modulus", "none"):
        xi, li = pr.ip(y, dists, _WL, _PX, 3, x0=x0, constraint=constraint)
        xf, lf = pr.fista(y, dists, _WL, _PX, outer=3, inner=4, tau=0.0, gamma=1.0, constraint=constraint,
                          x0=x0, accelerate=False)
        np.testing.assert_allclose(xi, xf, rtol=0, atol=1e-12)
        np.testing.assert_allclose(li, lf, rtol=1e-12, atol=1e-12 * li[0])
        assert li[1] < li[0]          # the start is not in the modulus set: the first step moves


def test_ip_sequential_order_differs_from_the_averaged_projection():
    """The reading for several distances: projections in turn. Averaging the
    distances' projections instead would be the gamma = 1/D step of Eq. (14);
    the two differ after one iteration."""
    truth, dists, Hs, y = _ip_problem(D=2, noise=True)
    xi, li = pr.ip(y, dists, _WL, _PX, 1)
    xa, _ = pr.fista(y, dists, _WL, _PX, outer=1, inner=2, tau=0.0, gamma=0.5, accelerate=False)
    # the trace holds F of Eq. (24) summed over both distances
    np.testing.assert_allclose(li[0], pr.data_term(pr.backprop(list(np.sqrt(y)), Hs), list(np.sqrt(y)), Hs),
                               rtol=1e-12)
    assert np.abs(xi - xa).max() > 1e-3
    # and the sequential order by hand: P_C(P_M2(P_C(P_M1 x0)))
    sy = np.sqrt(y)
    x = pr.backprop(list(sy), Hs)
    for s, H in zip(sy, Hs):
        u = pr.project_modulus(x, s, H)
        x = u / np.maximum(1.0, np.abs(u))
    np.testing.assert_allclose(xi, x, rtol=0, atol=1e-12)
