"""Independent real-valued constrained TV denoiser (test infrastructure only).

This is the real special case that Section IV-B of Gao & Cao generalises: the
fast gradient projection of Beck and Teboulle for min_{l <= x <= u}
0.5 ||x - b||^2 + lam TV(x) with the real isotropic (Eq. 3) or anisotropic
(Eq. 4) TV. It is written separately from ``oracle.tv`` (zero-padded dual
arrays, the divergence written in the "p + q - p_up - q_left" form, a box
projection) so that agreement between the two at equal iteration count pins the
complex solver's real reduction: for a real b, the complex type-I solver must
reproduce this with the same lam and the type-II solver with lam * alpha.
"""
import numpy as np


def _div(pp, qq):
    """Divergence-type operator on zero-padded duals.

    pp has shape (m+1, n) with rows 0 and m identically zero; row i+1 holds the
    vertical dual at row i. qq has shape (m, n+1) likewise along columns.
    Returns D[i,j] = p[i,j] - p[i-1,j] + q[i,j] - q[i,j-1].
    """
    return (pp[1:, :] - pp[:-1, :]) + (qq[:, 1:] - qq[:, :-1])


def _diffs(x, pp_shape, qq_shape):
    """Forward differences placed into zero-padded arrays (adjoint of _div)."""
    m, n = x.shape
    pp = np.zeros(pp_shape)
    qq = np.zeros(qq_shape)
    pp[1:m, :] = x[:-1, :] - x[1:, :]
    qq[:, 1:n] = x[:, :-1] - x[:, 1:]
    return pp, qq


def _project_dual(pp, qq, iso, radius):
    m = pp.shape[0] - 1
    n = qq.shape[1] - 1
    pp, qq = pp.copy(), qq.copy()
    if iso:
        # pixels with both differences: joint 2-norm ball
        P = pp[1:m, : n - 1]
        Q = qq[: m - 1, 1:n]
        nrm = np.sqrt(P ** 2 + Q ** 2)
        f = np.ones_like(nrm) if radius > 0 else np.zeros_like(nrm)
        big = nrm > radius
        f[big] = radius / nrm[big]
        pp[1:m, : n - 1] = P * f
        qq[: m - 1, 1:n] = Q * f
        # last column of p and last row of q: scalar boxes
        pp[1:m, n - 1:n] = np.clip(pp[1:m, n - 1:n], -radius, radius)
        qq[m - 1:m, 1:n] = np.clip(qq[m - 1:m, 1:n], -radius, radius)
    else:
        pp = np.clip(pp, -radius, radius)
        qq = np.clip(qq, -radius, radius)
    return pp, qq


def real_fgp(b, lam, K, iso=True, lo=-1.0, hi=1.0, radius=1.0, accelerate=True):
    """K iterations of the real constrained FGP (accelerate=False: the plain
    gradient projection); returns (x, p, q) where p, q are the unpadded
    vertical / horizontal duals.

    ``radius`` lets the same routine express a dual set scaled by alpha: with
    radius alpha and weight lam the iterates are alpha times those of radius 1
    and weight lam * alpha.
    """
    b = np.asarray(b, dtype=np.float64)
    m, n = b.shape
    ps, qs = (m + 1, n), (m, n + 1)
    p, q = np.zeros(ps), np.zeros(qs)
    p_old, q_old = p.copy(), q.copy()
    rp, rq = p.copy(), q.copy()
    t = 1.0
    step = 1.0 / (8.0 * lam)
    for _ in range(K):
        z = np.clip(b - lam * _div(rp, rq), lo, hi)
        dp, dq = _diffs(z, ps, qs)
        p, q = _project_dual(rp + step * dp, rq + step * dq, iso, radius)
        t_new = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0 if accelerate else 1.0
        c = (t - 1.0) / t_new
        rp = p + c * (p - p_old)
        rq = q + c * (q - q_old)
        p_old, q_old, t = p, q, t_new
    x = np.clip(b - lam * _div(p, q), lo, hi)
    return x, p[1:m, :], q[:, 1:n]
