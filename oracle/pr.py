"""FP64 phase-retrieval oracle (test infrastructure only).

Section V of Gao & Cao: free-space propagation by the angular spectrum method
(Eq. 23), the amplitude data-fidelity term F of Eq. (24) summed over several
propagation distances, its gradient (Eq. 27), and FISTA (Algorithm 1) with the
constrained-TV denoiser of ``oracle.tv`` as the proximity operator (Eq. 15 with
lam = tau * gamma).

Readings where the paper is silent:
  * frequencies f_x, f_y are numpy.fft.fftfreq(n, pixel) / (m, pixel) in the
    unshifted FFT order; evanescent frequencies (negative radicand) get H = 0;
  * F^{-1} is the exact inverse of F, so A_d is unitary on the propagating band;
  * z / |z| at z = 0 is taken as 1 (Appendix C allows any unit phasor there);
  * with several distances, F = sum_d F_d;
  * Algorithm 1's gradient point is z_k, and x_{k-1} at k = 1 is x_0;
  * gamma is fixed by default. The paper says gamma comes from a line search
    without naming one; ``line_search=True`` takes the backtracking rule of Beck
    and Teboulle's FISTA: keep the previous gamma, and shrink it by ``shrink``
    until F(x) <= F(z) + Re<grad F(z), x - z> + ||x - z||^2 / (2 gamma) holds for
    x = prox_{gamma R}(z - gamma grad F(z)), at most ``max_trials`` prox
    evaluations per outer iteration (the last one is accepted regardless);
  * each prox starts its dual from q = 0 (Algorithm 2, line 1); with
    ``warm_start=True`` it starts from the previous prox's last dual iterate,
    with the momentum restarted (r_1 = q_0, t_1 = 1).

The iterative projection baseline ``ip`` (Section VI-A) alternates the
measured-modulus projection of each distance, in turn, with P_C; with several
distances the paper is silent, and the sequential order is the reading taken
(averaging the distances' projections instead is exactly one step of the
proximal gradient iteration of Eq. 14 with tau = 0 and gamma = 1 / D).

Parity status: ``transfer``, ``A``, ``AH``, ``data_term`` and ``grad_F`` are
pinned by closed forms and finite differences. ``fista`` is pinned by Algorithm
1's closed form on a problem without measurements (y = 0, so F = (D/2)||x||^2 and
grad F = D x on a grid without evanescent frequencies; tau = 0, so the prox is
P_C): every iterate is a real multiple of x_0 given by a scalar recurrence, with
and without the modulus projection, with and without momentum, for one and
several distances, and the backtracking line search accepts exactly the steps
gamma <= 1 there. The paper prints no iterates of its own for a real problem.
``ip`` is pinned by the noise-free fixed point at the truth, idempotence of
each projection, the error-reduction inequality (with one distance F(x_k)
never increases) and, with one distance, its identity with one proximal
gradient step of step 1 whose prox is P_C alone.
"""
import numpy as np

from . import tv as _tv


def transfer(m, n, distance, wavelength, pixel):
    """H_d(f_x, f_y) = exp(i 2 pi d / lambda_s sqrt(1 - (lambda_s f_x)^2 - (lambda_s f_y)^2))."""
    fx = np.fft.fftfreq(n, d=pixel)[None, :]
    fy = np.fft.fftfreq(m, d=pixel)[:, None]
    arg = 1.0 - (wavelength * fx) ** 2 - (wavelength * fy) ** 2
    prop = arg > 0
    phase = 2.0 * np.pi / wavelength * distance * np.sqrt(np.where(prop, arg, 0.0))
    return np.where(prop, np.exp(1j * phase), 0.0)


def A(x, H):
    """Forward propagation, Eq. (23)."""
    return np.fft.ifft2(np.fft.fft2(x) * H)


def AH(z, H):
    """Adjoint of A: F^{-1}{ conj(H) F[z] } (F unitary up to the ifft scale)."""
    return np.fft.ifft2(np.fft.fft2(z) * np.conj(H))


def _phasor(z):
    a = np.abs(z)
    return np.where(a > 0, z / np.where(a > 0, a, 1.0), 1.0 + 0j), a


def data_term(x, sqrt_y, Hs):
    """F(x) = sum_d 0.5 || |A_d x| - sqrt(y_d) ||_F^2 (Eq. 24)."""
    return float(sum(0.5 * np.sum((np.abs(A(x, H)) - s) ** 2) for s, H in zip(sqrt_y, Hs)))


def grad_F(x, sqrt_y, Hs):
    """Eq. (27) summed over distances; the returned complex array holds the
    real-pair gradient (dF/du, dF/dv) as real + i imag."""
    g = np.zeros_like(np.asarray(x, dtype=np.complex128))
    for s, H in zip(sqrt_y, Hs):
        z = A(x, H)
        ph, a = _phasor(z)
        g = g + AH(ph * (a - s), H)
    return g


def backprop(sqrt_y, Hs):
    """Directly back-propagated field: (1/D) sum_d A_d^H sqrt(y_d)."""
    return sum(AH(s.astype(np.complex128), H) for s, H in zip(sqrt_y, Hs)) / len(Hs)


def fista(y, distances, wavelength, pixel, outer, inner, tau, gamma,
          kind="1i", alpha=0.5, constraint="modulus", x0=None, accelerate=True, inner_method="fgp",
          line_search=False, shrink=0.5, max_trials=20, warm_start=False, return_info=False):
    """Algorithm 1 with prox_{gamma R} = FGP (Algorithm 2) at lam = tau*gamma
    (inner_method="gp": the unaccelerated prox iteration of Eq. 21).

    y: (D, m, n) intensities. Returns (x_K, loss) where loss[k-1] = F(z_k), the
    data term at the k-th gradient point. accelerate=False gives the plain
    proximal gradient iteration of Eq. (14) (ISTA). With return_info, also a
    dict with the accepted step and the number of prox evaluations per outer
    iteration.
    """
    y = np.asarray(y, dtype=np.float64)
    D, m, n = y.shape
    Hs = [transfer(m, n, d, wavelength, pixel) for d in distances]
    sqrt_y = [np.sqrt(np.maximum(yy, 0.0)) for yy in y]
    x_prev = backprop(sqrt_y, Hs) if x0 is None else np.asarray(x0, dtype=np.complex128)
    z = x_prev.copy()
    t = 1.0
    loss, steps, trials = [], [], []
    q_warm = None
    for _ in range(outer):
        Fz = data_term(z, sqrt_y, Hs)
        loss.append(Fz)
        g = grad_F(z, sqrt_y, Hs)
        state = None if (not warm_start or q_warm is None) else (q_warm, q_warm, 0)
        for trial in range(max_trials if line_search else 1):
            x, (q, _, _) = _tv.fgp(z - gamma * g, tau * gamma, inner, kind, alpha, constraint, state=state,
                                   return_state=True, method=inner_method)
            if not line_search or trial == max_trials - 1:
                break
            d = x - z
            model = Fz + float(np.sum(g.real * d.real + g.imag * d.imag)) + float(np.sum(np.abs(d) ** 2)) / (2 * gamma)
            if data_term(x, sqrt_y, Hs) <= model:
                break
            gamma *= shrink
        steps.append(gamma)
        trials.append(trial + 1)
        q_warm = q
        t_new = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
        beta = (t - 1.0) / t_new if accelerate else 0.0
        z = x + beta * (x - x_prev)
        x_prev, t = x, t_new
    if return_info:
        return x_prev, np.array(loss), {"gamma": np.array(steps), "trials": np.array(trials)}
    return x_prev, np.array(loss)


def project_modulus(x, sqrt_y_d, H):
    """Nearest point of {x : |A_d x| = sqrt(y_d)} (A_d unitary on the grid):
    keep the phase of A_d x, impose the measured modulus, propagate back
    (unit phasor where A_d x = 0)."""
    ph, _ = _phasor(A(x, H))
    return AH(sqrt_y_d * ph, H)


def ip(y, distances, wavelength, pixel, iters, x0=None, constraint="modulus"):
    """The iterative projection (IP) comparison method of Section VI-A: the
    estimate is projected in turn onto the measured-modulus set of each
    distance, each projection followed by the projection P_C onto the
    nonnegative-absorption set of Eq. 25 (C = C^{m x n} for constraint="none").
    With one distance this is the classic alternation between the two sets.
    Starts from the back-propagated field unless x0 is given. Returns (x_K,
    loss) with loss[k] = F(x_k), the data term of Eq. (24) summed over d, at the
    start of iteration k + 1."""
    y = np.asarray(y, dtype=np.float64)
    D, m, n = y.shape
    Hs = [transfer(m, n, d, wavelength, pixel) for d in distances]
    sqrt_y = [np.sqrt(np.maximum(yy, 0.0)) for yy in y]
    x = backprop(sqrt_y, Hs) if x0 is None else np.asarray(x0, dtype=np.complex128)
    loss = []
    for _ in range(iters):
        loss.append(data_term(x, sqrt_y, Hs))
        for s, H in zip(sqrt_y, Hs):
            u = project_modulus(x, s, H)
            pu, pv = _tv.P_C(u.real, u.imag, constraint)
            x = pu + 1j * pv
    return x, np.array(loss)


def phase_rmse(x, truth):
    """Phase RMSE with the best global phase removed (Section VI-A)."""
    c = np.vdot(x, truth)
    rot = c / abs(c) if abs(c) > 0 else 1.0
    d = np.angle(x * rot * np.conj(truth))
    return float(np.sqrt(np.mean(d * d)))
