"""FP64 oracle: complex TV, projections and the FGP denoiser (test infrastructure).

Follows Gao & Cao, arXiv 2109.05496, Sections II and IV and Appendices A-B.
Shapes are the paper's, unpadded: for an m x n image, the vertical differences
live in (m-1) x n arrays and the horizontal ones in m x (n-1) arrays. A complex
image x = u + i v is handled as the real pair (u, v) (Section II, real-pair
representation). The dual variable is the 4-tuple q = (r1, r2, s1, s2): r pairs
with the real part u, s with the imaginary part v (Proposition 1).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline leg
may import this module.
"""
import numpy as np

KINDS = ("1i", "1a", "2i", "2a")
CONSTRAINTS = ("none", "modulus")


# ----------------------------------------------------------------------------
# Linear operators
# ----------------------------------------------------------------------------

def L(u):
    """Finite differences of one real plane, Eqs. (5)-(6).

    Returns (d1, d2) with d1[j,k] = u[j,k] - u[j+1,k]  (shape (m-1) x n) and
    d2[j,k] = u[j,k] - u[j,k+1]  (shape m x (n-1)).
    """
    u = np.asarray(u, dtype=np.float64)
    return u[:-1, :] - u[1:, :], u[:, :-1] - u[:, 1:]


def LT(a1, a2, shape):
    """Adjoint of ``L`` under the Frobenius inner product.

    The paper names this operator (Proposition 1) but never writes it out; it is
    the transpose of the difference map of Eqs. (5)-(6): each difference
    a1[j,k] (= u[j,k] - u[j+1,k]) sends +a1 to pixel (j,k) and -a1 to (j+1,k),
    and likewise for a2 along k.
    """
    m, n = shape
    z = np.zeros((m, n), dtype=np.float64)
    z[:-1, :] += a1
    z[1:, :] -= a1
    z[:, :-1] += a2
    z[:, 1:] -= a2
    return z


def L_pair(u, v):
    """p = (u1, u2, v1, v2) of a real pair (Section II notation)."""
    u1, u2 = L(u)
    v1, v2 = L(v)
    return (u1, u2, v1, v2)


def LT_pair(q, shape):
    """Adjoint of ``L_pair``: (r1, r2, s1, s2) -> (LT(r1, r2), LT(s1, s2))."""
    r1, r2, s1, s2 = q
    return LT(r1, r2, shape), LT(s1, s2, shape)


def zeros_dual(m, n):
    """q_0 of Algorithm 2, line 1."""
    return (np.zeros((m - 1, n)), np.zeros((m, n - 1)),
            np.zeros((m - 1, n)), np.zeros((m, n - 1)))


# ----------------------------------------------------------------------------
# Projections
# ----------------------------------------------------------------------------

def P_C(u, v, constraint="modulus", mask=None):
    """Projection onto C.

    constraint='modulus' is Eq. (25) with the projection of Eq. (26): each pixel
    divided by max{1, |x_jk|}. constraint='none' is C = C^{m x n} (the
    unconstrained "TV" model of Section VI-A), i.e. the identity. An optional
    0/1 support mask M further forces x_jk = 0 where M = 0; C stays a product
    of per-pixel convex sets, so its projection is M * (per-pixel projection).
    """
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    if constraint == "modulus":
        d = np.maximum(1.0, np.sqrt(u * u + v * v))
        u, v = u / d, v / d
    elif constraint != "none":
        raise ValueError(constraint)
    if mask is not None:
        mk = (np.asarray(mask) != 0).astype(np.float64)
        u, v = u * mk, v * mk
    return u, v


def _radial(x, y, rho):
    """rho * (x, y) / max(rho, ||(x, y)||); radius 0 projects to 0."""
    nrm = np.sqrt(x * x + y * y)
    den = np.maximum(rho, nrm)
    with np.errstate(invalid="ignore", divide="ignore"):
        f = np.where(den > 0, rho / np.where(den > 0, den, 1.0), 0.0)
    return x * f, y * f


def _scalar_clip(x, rho):
    """rho * x / max(rho, |x|); radius 0 projects to 0."""
    den = np.maximum(rho, np.abs(x))
    with np.errstate(invalid="ignore", divide="ignore"):
        f = np.where(den > 0, rho / np.where(den > 0, den, 1.0), 0.0)
    return x * f


def P_S(q, kind="1i", alpha=0.5):
    """Projection of the dual 4-tuple onto S for each TV kind.

    1i: Eq. (20) (set Eq. (17)); 1a: Eq. (33) (set Eq. (32));
    2i: Eq. (35) (set Eq. (34)); 2a: Eq. (37) (set Eq. (36)).
    Interior groups are (j, k) with j < m-1 and k < n-1 (0-based); the last
    column of r1/s1 and the last row of r2/s2 are the boundary groups.
    """
    r1, r2, s1, s2 = (np.array(a, dtype=np.float64, copy=True) for a in q)
    if kind == "1i":
        # interior: one 4-vector per pixel, radius 1
        a, b_, c, d = r1[:, :-1], r2[:-1, :], s1[:, :-1], s2[:-1, :]
        den = np.maximum(1.0, np.sqrt(a * a + b_ * b_ + c * c + d * d))
        r1[:, :-1], r2[:-1, :], s1[:, :-1], s2[:-1, :] = a / den, b_ / den, c / den, d / den
        # last column of the vertical pair, last row of the horizontal pair
        den = np.maximum(1.0, np.sqrt(r1[:, -1:] ** 2 + s1[:, -1:] ** 2))
        r1[:, -1:], s1[:, -1:] = r1[:, -1:] / den, s1[:, -1:] / den
        den = np.maximum(1.0, np.sqrt(r2[-1:, :] ** 2 + s2[-1:, :] ** 2))
        r2[-1:, :], s2[-1:, :] = r2[-1:, :] / den, s2[-1:, :] / den
    elif kind == "1a":
        den = np.maximum(1.0, np.sqrt(r1 * r1 + s1 * s1))
        r1, s1 = r1 / den, s1 / den
        den = np.maximum(1.0, np.sqrt(r2 * r2 + s2 * s2))
        r2, s2 = r2 / den, s2 / den
    elif kind == "2i":
        ra, sa = alpha, 1.0 - alpha
        # interior: (r1, r2) in the alpha-ball, (s1, s2) in the (1-alpha)-ball
        r1[:, :-1], r2[:-1, :] = _radial(r1[:, :-1], r2[:-1, :], ra)
        s1[:, :-1], s2[:-1, :] = _radial(s1[:, :-1], s2[:-1, :], sa)
        r1[:, -1:] = _scalar_clip(r1[:, -1:], ra)
        s1[:, -1:] = _scalar_clip(s1[:, -1:], sa)
        r2[-1:, :] = _scalar_clip(r2[-1:, :], ra)
        s2[-1:, :] = _scalar_clip(s2[-1:, :], sa)
    elif kind == "2a":
        r1, r2 = _scalar_clip(r1, alpha), _scalar_clip(r2, alpha)
        s1, s2 = _scalar_clip(s1, 1.0 - alpha), _scalar_clip(s2, 1.0 - alpha)
    else:
        raise ValueError(kind)
    return (r1, r2, s1, s2)


# ----------------------------------------------------------------------------
# TV seminorms, Eqs. (3), (4), (7)-(10)
# ----------------------------------------------------------------------------

def tv_real(u, iso=True):
    """Real TV: isotropic Eq. (3), anisotropic Eq. (4)."""
    u = np.asarray(u, dtype=np.float64)
    m, n = u.shape
    tot = 0.0
    for j in range(m):
        for k in range(n):
            dv = u[j, k] - u[j + 1, k] if j + 1 < m else None
            dh = u[j, k] - u[j, k + 1] if k + 1 < n else None
            if dv is not None and dh is not None:
                tot += np.sqrt(dv * dv + dh * dh) if iso else abs(dv) + abs(dh)
            elif dv is not None:
                tot += abs(dv)
            elif dh is not None:
                tot += abs(dh)
    return tot


def tv(x, kind="1i", alpha=0.5):
    """Complex TV of x (complex array) per Eqs. (7)-(10), written in the
    complex-modulus form of each definition's first line."""
    x = np.asarray(x, dtype=np.complex128)
    if kind in ("2i", "2a"):
        iso = kind == "2i"
        return alpha * tv_vec(x.real, iso) + (1.0 - alpha) * tv_vec(x.imag, iso)
    dv = x[:-1, :] - x[1:, :]            # complex vertical differences
    dh = x[:, :-1] - x[:, 1:]
    av, ah = np.abs(dv), np.abs(dh)
    if kind == "1i":
        inner = np.sqrt(av[:, :-1] ** 2 + ah[:-1, :] ** 2).sum()
    elif kind == "1a":
        inner = (av[:, :-1] + ah[:-1, :]).sum()
    else:
        raise ValueError(kind)
    return inner + av[:, -1:].sum() + ah[-1:, :].sum()


def tv_vec(u, iso=True):
    """Vectorised Eq. (3) / (4) for a real plane (tv_real is the loop form)."""
    u = np.asarray(u, dtype=np.float64)
    dv = u[:-1, :] - u[1:, :]
    dh = u[:, :-1] - u[:, 1:]
    if iso:
        inner = np.sqrt(dv[:, :-1] ** 2 + dh[:-1, :] ** 2).sum()
    else:
        inner = (np.abs(dv[:, :-1]) + np.abs(dh[:-1, :])).sum()
    return inner + np.abs(dv[:, -1:]).sum() + np.abs(dh[-1:, :]).sum()


# ----------------------------------------------------------------------------
# FGP, Algorithm 2
# ----------------------------------------------------------------------------

def t_sequence(K):
    """t_1 = 1, t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2 (Algorithm 2, line 4).
    Returns t[0..K+1] with t[k] = t_k (t[0] unused)."""
    t = np.zeros(K + 2)
    t[1] = 1.0
    for k in range(1, K + 1):
        t[k + 1] = (1.0 + np.sqrt(1.0 + 4.0 * t[k] * t[k])) / 2.0
    return t


def _dual_add(a, b, s=1.0):
    return tuple(x + s * y for x, y in zip(a, b))


def grad_h(rq, b, lam, constraint="modulus", mask=None):
    """Gradient of the dual objective, Eq. (19): -2 lam L(P_C(b - lam L^T q))."""
    m, n = b.shape
    lu, lv = LT_pair(rq, (m, n))
    yu, yv = P_C(b.real - lam * lu, b.imag - lam * lv, constraint, mask)
    return tuple(-2.0 * lam * d for d in L_pair(yu, yv))


def primal_from_dual(q, b, lam, constraint="modulus", mask=None):
    """x = P_C(b - lam L^T q), Eq. (18); returns a complex array."""
    m, n = b.shape
    lu, lv = LT_pair(q, (m, n))
    yu, yv = P_C(b.real - lam * lu, b.imag - lam * lv, constraint, mask)
    return yu + 1j * yv


def fgp(b, lam, K, kind="1i", alpha=0.5, constraint="modulus", mask=None,
        state=None, return_state=False, method="fgp"):
    """Algorithm 2 followed by Eq. (18); method="gp" runs the basic gradient
    projection of Eq. (21) instead (the same step with no extrapolation).

    b: complex array (upcast to complex128). Runs K iterations. ``state`` =
    (q_k, q_{k-1}, k) resumes from iteration k (t_k follows from k alone).
    Returns x (complex128); with return_state, also (q_K', q_{K'-1}, K').

    lam = 0 makes the step 1/(16 lam^2) undefined while the TV term vanishes, so
    the exact solution P_C(b) is returned; K = 0 gives P_C(b) by Eq. (18) with
    q = 0.
    """
    b = np.asarray(b, dtype=np.complex128)
    m, n = b.shape
    if state is None:
        q, q_prev, k0 = zeros_dual(m, n), zeros_dual(m, n), 0
    else:
        q, q_prev, k0 = state
    if lam == 0:
        yu, yv = P_C(b.real, b.imag, constraint, mask)
        x = yu + 1j * yv
        return (x, (q, q_prev, k0 + K)) if return_state else x
    if method not in ("fgp", "gp"):
        raise ValueError(method)
    t = t_sequence(k0 + K + 1)
    if method == "gp":
        t[:] = 1.0                          # Eq. (21): r_k = q_{k-1}
    # r_{k0+1} = q_{k0} + ((t_{k0} - 1)/t_{k0+1}) (q_{k0} - q_{k0-1}); at k0 = 0 it is q_0.
    beta = (t[k0] - 1.0) / t[k0 + 1] if k0 >= 1 else 0.0
    r = tuple(a + beta * (a - c) for a, c in zip(q, q_prev))
    inv_L = 1.0 / (16.0 * lam * lam)          # step 1/(16 lam^2), Section IV-B
    for k in range(k0 + 1, k0 + K + 1):
        gh = grad_h(r, b, lam, constraint, mask)
        q_new = P_S(_dual_add(r, gh, -inv_L), kind, alpha)          # line 3
        beta = (t[k] - 1.0) / t[k + 1]                                # lines 4-5
        r = tuple(a + beta * (a - c) for a, c in zip(q_new, q))
        q_prev, q = q, q_new
    x = primal_from_dual(q, b, lam, constraint, mask)
    return (x, (q, q_prev, k0 + K)) if return_state else x


# ----------------------------------------------------------------------------
# Objective, dual function and duality gap
# ----------------------------------------------------------------------------

def primal_objective(x, b, lam, kind="1i", alpha=0.5):
    """Eq. (1) for x in C: 0.5 ||x - b||_F^2 + lam ||x||_TV."""
    x = np.asarray(x, dtype=np.complex128)
    return 0.5 * np.sum(np.abs(x - b) ** 2) + lam * tv(x, kind, alpha)


def dual_value(q, b, lam, constraint="modulus", mask=None):
    """Dual function of Eq. (15) at q in S, from Proposition 1 / Appendix A:
    D(q) = 0.5 (||b||^2 - h(q)), h(q) = ||w||^2 - ||H_C(w)||^2, w = b - lam L^T q.
    (The scaling by 1/lam of Appendix A is undone so that D bounds Eq. (1).)"""
    b = np.asarray(b, dtype=np.complex128)
    m, n = b.shape
    lu, lv = LT_pair(q, (m, n))
    wu, wv = b.real - lam * lu, b.imag - lam * lv
    pu, pv = P_C(wu, wv, constraint, mask)
    h = np.sum(wu ** 2 + wv ** 2) - np.sum((wu - pu) ** 2 + (wv - pv) ** 2)
    return 0.5 * (np.sum(np.abs(b) ** 2) - h)


def gap_primal_minus_dual(q, b, lam, kind="1i", alpha=0.5, constraint="modulus", mask=None):
    """P(x(q)) - D(q) with x(q) from Eq. (18)."""
    x = primal_from_dual(q, b, lam, constraint, mask)
    return primal_objective(x, b, lam, kind, alpha) - dual_value(q, b, lam, constraint, mask)


def gap_groups(q, b, lam, kind="1i", alpha=0.5, constraint="modulus", mask=None):
    """The same gap as a sum of per-group nonnegative terms:
    lam * sum_groups (||(L x)_g||_* - <q_g, (L x)_g>), x = x(q).

    Since D(q) = 0.5||x-b||^2 + lam <q, L x> at x = x(q) (Appendix A with the
    infimum attained at Eq. (18)), P - D = lam (TV(x) - <q, L x>), and each
    group's term is >= 0 by Cauchy-Schwarz when q lies in S.
    Returns (total, per_group_min)."""
    x = primal_from_dual(q, b, lam, constraint, mask)
    return gap_at(x, q, lam, kind, alpha)


def gap_at(x, q, lam, kind="1i", alpha=0.5):
    """lam * sum_groups (||(L x)_g||_* - <q_g, (L x)_g>) for a given primal x
    and dual q (the group sum of gap_groups without forming x(q)).
    Returns (total, per_group_min)."""
    x = np.asarray(x, dtype=np.complex128)
    u1, u2, v1, v2 = L_pair(x.real, x.imag)
    r1, r2, s1, s2 = q
    terms = []
    if kind == "1i":
        terms.append(np.sqrt(u1[:, :-1] ** 2 + u2[:-1, :] ** 2 + v1[:, :-1] ** 2 + v2[:-1, :] ** 2)
                     - (r1[:, :-1] * u1[:, :-1] + r2[:-1, :] * u2[:-1, :]
                        + s1[:, :-1] * v1[:, :-1] + s2[:-1, :] * v2[:-1, :]))
        terms.append(np.sqrt(u1[:, -1:] ** 2 + v1[:, -1:] ** 2) - (r1[:, -1:] * u1[:, -1:] + s1[:, -1:] * v1[:, -1:]))
        terms.append(np.sqrt(u2[-1:, :] ** 2 + v2[-1:, :] ** 2) - (r2[-1:, :] * u2[-1:, :] + s2[-1:, :] * v2[-1:, :]))
    elif kind == "1a":
        terms.append(np.sqrt(u1 ** 2 + v1 ** 2) - (r1 * u1 + s1 * v1))
        terms.append(np.sqrt(u2 ** 2 + v2 ** 2) - (r2 * u2 + s2 * v2))
    elif kind == "2i":
        a, c = alpha, 1.0 - alpha
        terms.append(a * np.sqrt(u1[:, :-1] ** 2 + u2[:-1, :] ** 2) - (r1[:, :-1] * u1[:, :-1] + r2[:-1, :] * u2[:-1, :]))
        terms.append(c * np.sqrt(v1[:, :-1] ** 2 + v2[:-1, :] ** 2) - (s1[:, :-1] * v1[:, :-1] + s2[:-1, :] * v2[:-1, :]))
        terms.append(a * np.abs(u1[:, -1:]) - r1[:, -1:] * u1[:, -1:])
        terms.append(c * np.abs(v1[:, -1:]) - s1[:, -1:] * v1[:, -1:])
        terms.append(a * np.abs(u2[-1:, :]) - r2[-1:, :] * u2[-1:, :])
        terms.append(c * np.abs(v2[-1:, :]) - s2[-1:, :] * v2[-1:, :])
    elif kind == "2a":
        a, c = alpha, 1.0 - alpha
        for d, r in ((u1, r1), (u2, r2)):
            terms.append(a * np.abs(d) - r * d)
        for d, s in ((v1, s1), (v2, s2)):
            terms.append(c * np.abs(d) - s * d)
    else:
        raise ValueError(kind)
    total = lam * sum(float(t.sum()) for t in terms)
    mins = [float(t.min()) for t in terms if t.size]
    return total, (min(mins) if mins else 0.0)
