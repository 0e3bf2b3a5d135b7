"""Reverse-mode derivative of the K-step FGP map (test infrastructure only).

The map is (b, lam) -> x_K of Algorithm 2 followed by Eq. (18). The paper does
not differentiate it; this is the chain rule taken over the algorithm's steps:

    r_k = q_{k-1} + beta_{k-1} (q_{k-1} - q_{k-2})      (line 5, beta_0 = 0)
    w_k = b - lam L^T r_k,  y_k = P_C(w_k)               (Eq. 19's inner part)
    g_k = r_k + L y_k / (8 lam)                          (line 3 with Eq. 19 and 16 lam^2)
    q_k = P_S(g_k)
    x   = P_C(b - lam L^T q_K)                           (Eq. 18)

Complex gradients use the real-pair convention dl/du + i dl/dv (the
representation of Section II), which is what PyTorch returns for a real loss of
a complex tensor.

Non-smooth points: a ball projection v -> rho v / max(rho, ||v||) is given the
identity Jacobian when ||v|| <= rho and rho (I - v v^T/||v||^2)/||v|| when
||v|| > rho; a zero radius gives the zero map and the zero Jacobian. P_C uses
the same rule with rho = 1 (masked pixels have zero Jacobian).

``fgp_vjp`` is the hand-written reverse pass (numpy, float64).
``torch_fgp`` is an independently written unrolled forward in torch float64
whose autograd serves as a second reference.
"""
import numpy as np

from . import tv as _tv


def _ball_vjp(vecs, bars, rho):
    """J^T bar for the projection of the stacked vectors ``vecs`` (list of
    equally shaped arrays forming one vector per position) onto the ball of
    radius rho; J is symmetric so J^T = J."""
    n2 = sum(v * v for v in vecs)
    if rho <= 0:
        return [np.zeros_like(b) for b in bars]
    nrm = np.sqrt(n2)
    out_side = nrm > rho
    safe = np.where(out_side, nrm, 1.0)
    dot = sum(v * b for v, b in zip(vecs, bars)) / (safe * safe)
    res = []
    for v, b in zip(vecs, bars):
        scaled = rho * (b - v * dot) / safe
        res.append(np.where(out_side, scaled, b))
    return res


def PS_vjp(g, gbar, kind, alpha):
    """J_{P_S}(g)^T gbar for the four kinds (Eqs. 20, 33, 35, 37)."""
    r1, r2, s1, s2 = g
    a1, a2, c1, c2 = (np.array(x, dtype=np.float64, copy=True) for x in gbar)
    o1, o2, p1, p2 = a1.copy(), a2.copy(), c1.copy(), c2.copy()
    if kind == "1i":
        I1, I2 = (slice(None), slice(None, -1)), (slice(None, -1), slice(None))
        res = _ball_vjp([r1[I1], r2[I2], s1[I1], s2[I2]], [a1[I1], a2[I2], c1[I1], c2[I2]], 1.0)
        o1[I1], o2[I2], p1[I1], p2[I2] = res
        B1, B2 = (slice(None), slice(-1, None)), (slice(-1, None), slice(None))
        o1[B1], p1[B1] = _ball_vjp([r1[B1], s1[B1]], [a1[B1], c1[B1]], 1.0)
        o2[B2], p2[B2] = _ball_vjp([r2[B2], s2[B2]], [a2[B2], c2[B2]], 1.0)
    elif kind == "1a":
        o1, p1 = _ball_vjp([r1, s1], [a1, c1], 1.0)
        o2, p2 = _ball_vjp([r2, s2], [a2, c2], 1.0)
    elif kind == "2i":
        ra, sa = alpha, 1.0 - alpha
        I1, I2 = (slice(None), slice(None, -1)), (slice(None, -1), slice(None))
        o1[I1], o2[I2] = _ball_vjp([r1[I1], r2[I2]], [a1[I1], a2[I2]], ra)
        p1[I1], p2[I2] = _ball_vjp([s1[I1], s2[I2]], [c1[I1], c2[I2]], sa)
        B1, B2 = (slice(None), slice(-1, None)), (slice(-1, None), slice(None))
        (o1[B1],) = _ball_vjp([r1[B1]], [a1[B1]], ra)
        (p1[B1],) = _ball_vjp([s1[B1]], [c1[B1]], sa)
        (o2[B2],) = _ball_vjp([r2[B2]], [a2[B2]], ra)
        (p2[B2],) = _ball_vjp([s2[B2]], [c2[B2]], sa)
    elif kind == "2a":
        (o1,) = _ball_vjp([r1], [a1], alpha)
        (o2,) = _ball_vjp([r2], [a2], alpha)
        (p1,) = _ball_vjp([s1], [c1], 1.0 - alpha)
        (p2,) = _ball_vjp([s2], [c2], 1.0 - alpha)
    else:
        raise ValueError(kind)
    return (o1, o2, p1, p2)


def PC_vjp(wu, wv, bu, bv, constraint, mask):
    if constraint == "modulus":
        ou, ov = _ball_vjp([wu, wv], [bu, bv], 1.0)
    else:
        ou, ov = bu.copy(), bv.copy()
    if mask is not None:
        mk = (np.asarray(mask) != 0).astype(np.float64)
        ou, ov = ou * mk, ov * mk
    return ou, ov


def _inner(a, b):
    return float(sum(np.sum(x * y) for x, y in zip(a, b)))


def fgp_vjp(b, lam, K, xbar, kind="1i", alpha=0.5, constraint="modulus", mask=None, method="fgp"):
    """Returns (x, bbar complex, lambar float) for loss gradient xbar (complex,
    real-pair convention)."""
    b = np.asarray(b, dtype=np.complex128)
    xbar = np.asarray(xbar, dtype=np.complex128)
    m, n = b.shape
    if lam == 0 or K == 0:
        pu, pv = _tv.P_C(b.real, b.imag, constraint, mask)
        bu, bv = PC_vjp(b.real, b.imag, xbar.real, xbar.imag, constraint, mask)
        return pu + 1j * pv, bu + 1j * bv, 0.0
    t = _tv.t_sequence(K + 1)
    beta = np.zeros(K + 1)              # beta[k] = (t_k - 1)/t_{k+1}, beta[0] = 0
    if method == "fgp":
        for k in range(1, K + 1):
            beta[k] = (t[k] - 1.0) / t[k + 1]
    c = 1.0 / (8.0 * lam)
    # forward, keeping every iterate
    qs = [_tv.zeros_dual(m, n)]
    rs, ws, ys, gs = [None], [None], [None], [None]
    for k in range(1, K + 1):
        if k == 1:
            r = qs[0]
        else:
            r = tuple(a + beta[k - 1] * (a - z) for a, z in zip(qs[k - 1], qs[k - 2]))
        lu, lv = _tv.LT_pair(r, (m, n))
        wu, wv = b.real - lam * lu, b.imag - lam * lv
        yu, yv = _tv.P_C(wu, wv, constraint, mask)
        g = tuple(a + c * d for a, d in zip(r, _tv.L_pair(yu, yv)))
        q = _tv.P_S(g, kind, alpha)
        rs.append(r); ws.append((wu, wv)); ys.append((yu, yv)); gs.append(g); qs.append(q)
    lu, lv = _tv.LT_pair(qs[K], (m, n))
    ou, ov = b.real - lam * lu, b.imag - lam * lv
    xu, xv = _tv.P_C(ou, ov, constraint, mask)
    # reverse
    wbu, wbv = PC_vjp(ou, ov, xbar.real, xbar.imag, constraint, mask)
    bbu, bbv = wbu.copy(), wbv.copy()
    lambar = -(np.sum(wbu * lu) + np.sum(wbv * lv))
    qbar = [tuple(np.zeros_like(a) for a in qs[0]) for _ in range(K + 1)]
    qbar[K] = tuple(-lam * d for d in _tv.L_pair(wbu, wbv))
    for k in range(K, 0, -1):
        gbar = PS_vjp(gs[k], qbar[k], kind, alpha)
        rbar = [a.copy() for a in gbar]
        ybu, ybv = _tv.LT_pair(gbar, (m, n))
        ybu, ybv = c * ybu, c * ybv
        lambar += -_inner(gbar, _tv.L_pair(*ys[k])) / (8.0 * lam * lam)
        wbu, wbv = PC_vjp(ws[k][0], ws[k][1], ybu, ybv, constraint, mask)
        bbu += wbu
        bbv += wbv
        lr = _tv.LT_pair(rs[k], (m, n))
        lambar += -(np.sum(wbu * lr[0]) + np.sum(wbv * lr[1]))
        for i, d in enumerate(_tv.L_pair(wbu, wbv)):
            rbar[i] = rbar[i] - lam * d
        if k >= 2:
            bk = beta[k - 1]
            qbar[k - 1] = tuple(a + (1.0 + bk) * d for a, d in zip(qbar[k - 1], rbar))
            qbar[k - 2] = tuple(a - bk * d for a, d in zip(qbar[k - 2], rbar))
        # k == 1: r_1 = q_0 is a constant
    return xu + 1j * xv, bbu + 1j * bbv, float(lambar)


# ----------------------------------------------------------------------------
# Independent torch float64 forward (autograd reference)
# ----------------------------------------------------------------------------

def torch_fgp(b_re, b_im, lam, K, kind="1i", alpha=0.5, constraint="modulus", mask=None):
    """Unrolled FGP in torch float64 on zero-padded m x n dual planes.

    Written without ``oracle.tv``: padded duals P1 (vertical, last row zero) and
    P2 (horizontal, last column zero) per real/imaginary plane, differences by
    tensor slicing, projections by torch.where on squared norms (so that a zero
    vector has a finite gradient). Returns (x_re, x_im) tensors.
    """
    import torch
    m, n = b_re.shape
    dt = b_re.dtype
    mk = None if mask is None else torch.as_tensor((np.asarray(mask) != 0).astype(np.float64), dtype=dt)
    rowpad = torch.ones((m, n), dtype=dt)
    rowpad[-1, :] = 0.0
    colpad = torch.ones((m, n), dtype=dt)
    colpad[:, -1] = 0.0

    def grad_op(y):
        d1 = torch.zeros_like(y)
        d2 = torch.zeros_like(y)
        d1 = torch.cat([y[:-1, :] - y[1:, :], torch.zeros((1, n), dtype=dt)], 0)
        d2 = torch.cat([y[:, :-1] - y[:, 1:], torch.zeros((m, 1), dtype=dt)], 1)
        return d1, d2

    def div_op(p1, p2):
        up = torch.cat([torch.zeros((1, n), dtype=dt), p1[:-1, :]], 0)
        left = torch.cat([torch.zeros((m, 1), dtype=dt), p2[:, :-1]], 1)
        return p1 - up + p2 - left

    def ball(vs, rho):
        if rho <= 0:
            return [v * 0.0 for v in vs]
        n2 = sum(v * v for v in vs)
        out = n2 > rho * rho
        safe = torch.where(out, n2, torch.ones_like(n2))
        f = torch.where(out, rho / torch.sqrt(safe), torch.ones_like(n2))
        return [v * f for v in vs]

    def proj_C(u, v):
        if constraint == "modulus":
            u, v = ball([u, v], 1.0)
        if mk is not None:
            u, v = u * mk, v * mk
        return u, v

    interior = rowpad * colpad
    lastcol = rowpad * (1 - colpad)     # rows < m-1, column n-1: only P1 exists
    lastrow = colpad * (1 - rowpad)     # row m-1, columns < n-1: only P2 exists

    def proj_S(R1, R2, S1, S2):
        if kind == "1i":
            a = ball([R1, R2, S1, S2], 1.0)
            e1 = ball([R1, S1], 1.0)
            e2 = ball([R2, S2], 1.0)
            R1n = interior * a[0] + lastcol * e1[0]
            S1n = interior * a[2] + lastcol * e1[1]
            R2n = interior * a[1] + lastrow * e2[0]
            S2n = interior * a[3] + lastrow * e2[1]
            return R1n, R2n, S1n, S2n
        if kind == "1a":
            R1n, S1n = ball([R1, S1], 1.0)
            R2n, S2n = ball([R2, S2], 1.0)
            return R1n, R2n, S1n, S2n
        if kind == "2i":
            ra, sa = alpha, 1.0 - alpha
            ar = ball([R1, R2], ra)
            asv = ball([S1, S2], sa)
            R1n = interior * ar[0] + lastcol * ball([R1], ra)[0]
            S1n = interior * asv[0] + lastcol * ball([S1], sa)[0]
            R2n = interior * ar[1] + lastrow * ball([R2], ra)[0]
            S2n = interior * asv[1] + lastrow * ball([S2], sa)[0]
            return R1n, R2n, S1n, S2n
        if kind == "2a":
            return (ball([R1], alpha)[0], ball([R2], alpha)[0],
                    ball([S1], 1.0 - alpha)[0], ball([S2], 1.0 - alpha)[0])
        raise ValueError(kind)

    if (not isinstance(lam, torch.Tensor) and lam == 0) or K == 0:
        return proj_C(b_re, b_im)
    z = torch.zeros((m, n), dtype=dt)
    Q = (z, z, z, z)
    Qp = Q
    t = 1.0
    step = 1.0 / (8.0 * lam)
    R = Q
    for _ in range(K):
        wu = b_re - lam * div_op(R[0], R[1])
        wv = b_im - lam * div_op(R[2], R[3])
        yu, yv = proj_C(wu, wv)
        du1, du2 = grad_op(yu)
        dv1, dv2 = grad_op(yv)
        G = (R[0] + step * du1 * rowpad, R[1] + step * du2 * colpad,
             R[2] + step * dv1 * rowpad, R[3] + step * dv2 * colpad)
        Qn = proj_S(*G)
        t_new = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
        beta = (t - 1.0) / t_new
        R = tuple(a + beta * (a - c) for a, c in zip(Qn, Q))
        Qp, Q, t = Q, Qn, t_new
    return proj_C(b_re - lam * div_op(Q[0], Q[1]), b_im - lam * div_op(Q[2], Q[3]))
