"""Dense-matrix brute-force solver for tiny complex TV problems (test
infrastructure only).

Solves Eq. (1), min_{x in C} 0.5 ||x - b||^2 + lam ||x||_TV, for a few-pixel
image with the accelerated primal-dual method of Chambolle and Pock for a
1-strongly convex primal term. Nothing is shared with ``oracle.tv``: the
difference operator is an explicit dense matrix built entry by entry from
Eqs. (5)-(6), and the TV groups are read off Eqs. (7)-(10) directly.

``certificate`` evaluates P(x) - D(y) for any primal x in C and dual y in lam*S
with these dense objects. Because P is 1-strongly convex and D(y) <= P(x*),
0.5 ||x - x*||^2 <= P(x) - D(y): the certificate bounds the distance of x to
the unique minimiser whichever solver produced x.
"""
import numpy as np


def difference_matrix(m, n):
    """Rows: u1 (vertical, (m-1) x n, row-major), u2 (horizontal, m x (n-1)),
    then v1, v2. Columns: u (m*n, row-major) then v. Returns (D, index dict)."""
    N = m * n
    rows = []
    idx = {}
    for plane, off in (("u", 0), ("v", N)):
        for j in range(m - 1):
            for k in range(n):
                r = np.zeros(2 * N)
                r[off + j * n + k] = 1.0
                r[off + (j + 1) * n + k] = -1.0
                idx[(plane, 1, j, k)] = len(rows)
                rows.append(r)
        for j in range(m):
            for k in range(n - 1):
                r = np.zeros(2 * N)
                r[off + j * n + k] = 1.0
                r[off + j * n + k + 1] = -1.0
                idx[(plane, 2, j, k)] = len(rows)
                rows.append(r)
    D = np.array(rows) if rows else np.zeros((0, 2 * N))
    return D, idx


def tv_groups(m, n, kind, alpha):
    """List of (row indices into D x, weight) such that
    TV(x) = sum_g weight_g * ||(D x)[rows_g]||_2, read off Eqs. (7)-(10)."""
    _, idx = difference_matrix(m, n)
    groups = []

    def has(p, d, j, k):
        return (p, d, j, k) in idx

    for j in range(m):
        for k in range(n):
            if kind == "1i":
                g = [idx[(p, d, j, k)] for d in (1, 2) for p in ("u", "v") if has(p, d, j, k)]
                if g:
                    groups.append((g, 1.0))
            elif kind == "1a":
                for d in (1, 2):
                    g = [idx[(p, d, j, k)] for p in ("u", "v") if has(p, d, j, k)]
                    if g:
                        groups.append((g, 1.0))
            elif kind == "2i":
                for p, w in (("u", alpha), ("v", 1.0 - alpha)):
                    g = [idx[(p, d, j, k)] for d in (1, 2) if has(p, d, j, k)]
                    if g:
                        groups.append((g, w))
            elif kind == "2a":
                for p, w in (("u", alpha), ("v", 1.0 - alpha)):
                    for d in (1, 2):
                        if has(p, d, j, k):
                            groups.append(([idx[(p, d, j, k)]], w))
            else:
                raise ValueError(kind)
    return groups


class Problem:
    """Dense form of Eq. (1) for one tiny image."""

    def __init__(self, b, lam, kind="1i", alpha=0.5, constraint="modulus", mask=None):
        b = np.asarray(b, dtype=np.complex128)
        self.m, self.n = m, n = b.shape
        self.N = m * n
        self.lam = float(lam)
        self.constraint = constraint
        self.D, _ = difference_matrix(m, n)
        groups = tv_groups(m, n, kind, alpha)
        P = self.D.shape[0]
        width = max([len(g) for g, _ in groups], default=1)
        # padded group table; index P points at an always-zero slot
        self.gidx = np.full((len(groups), width), P, dtype=np.int64)
        for i, (g, _) in enumerate(groups):
            self.gidx[i, :len(g)] = g
        self.gw = np.array([w for _, w in groups])
        self.bvec = np.concatenate([b.real.ravel(), b.imag.ravel()])
        self.mvec = np.ones(self.N) if mask is None else (np.asarray(mask).ravel() != 0).astype(float)

    def proj_C(self, z):
        N = self.N
        u, v = z[:N], z[N:]
        if self.constraint == "modulus":
            d = np.maximum(1.0, np.hypot(u, v))
            u, v = u / d, v / d
        return np.concatenate([u * self.mvec, v * self.mvec])

    def tv(self, xv):
        p = np.append(self.D @ xv, 0.0)
        return float(np.sum(self.gw * np.sqrt(np.sum(p[self.gidx] ** 2, axis=1))))

    def primal(self, xv):
        return 0.5 * np.sum((xv - self.bvec) ** 2) + self.lam * self.tv(xv)

    def dual(self, yv):
        """min_{x in C} 0.5||x-b||^2 + <y, D x>, attained at P_C(b - D^T y)."""
        xv = self.proj_C(self.bvec - self.D.T @ yv)
        return 0.5 * np.sum((xv - self.bvec) ** 2) + yv @ (self.D @ xv)

    def proj_dual(self, yv):
        """Projection onto lam * S (group g: ball of radius lam * weight_g)."""
        ye = np.append(yv, 0.0)
        nr = np.sqrt(np.sum(ye[self.gidx] ** 2, axis=1))
        rad = self.lam * self.gw
        f = np.where(nr > rad, rad / np.where(nr > 0, nr, 1.0), 1.0)
        f = np.where(rad <= 0, 0.0, f)
        out = ye.copy()
        out[self.gidx] = ye[self.gidx] * f[:, None]
        out[-1] = 0.0
        return out[:-1]

    def in_dual_set(self, yv, tol=1e-12):
        ye = np.append(yv, 0.0)
        nr = np.sqrt(np.sum(ye[self.gidx] ** 2, axis=1))
        return bool(np.all(nr <= self.lam * self.gw * (1 + tol) + tol))

    def certificate(self, xv, yv):
        """P(x) - D(y); requires x in C and y in lam*S."""
        return self.primal(xv) - self.dual(yv)


def to_vec(x):
    x = np.asarray(x, dtype=np.complex128)
    return np.concatenate([x.real.ravel(), x.imag.ravel()])


def dual_to_vec(q, lam):
    """(r1, r2, s1, s2) unpadded arrays -> lam * (u1, u2, v1, v2 rows of D)."""
    r1, r2, s1, s2 = q
    return lam * np.concatenate([np.ravel(r1), np.ravel(r2), np.ravel(s1), np.ravel(s2)])


def solve(b, lam, kind="1i", alpha=0.5, constraint="modulus", mask=None, iters=40000):
    """Accelerated primal-dual iterations. Returns (x, y, certificate)."""
    pr = Problem(b, lam, kind, alpha, constraint, mask)
    m, n, N = pr.m, pr.n, pr.N
    D = pr.D
    x = pr.proj_C(pr.bvec)
    y = np.zeros(D.shape[0])
    if D.shape[0] == 0 or lam == 0:
        return x[:N].reshape(m, n) + 1j * x[N:].reshape(m, n), y, 0.0
    tau = sigma = 1.0 / np.linalg.norm(D, 2)
    xbar = x.copy()
    for _ in range(iters):
        y = pr.proj_dual(y + sigma * (D @ xbar))
        z = x - tau * (D.T @ y)
        x_new = pr.proj_C((tau * pr.bvec + z) / (1.0 + tau))   # prox of 0.5||.-b||^2 + I_C
        theta = 1.0 / np.sqrt(1.0 + 2.0 * tau)
        tau, sigma = theta * tau, sigma / theta
        xbar = x_new + theta * (x_new - x)
        x = x_new
    cert = pr.certificate(x, y)
    return x[:N].reshape(m, n) + 1j * x[N:].reshape(m, n), y, cert
