"""Property-based checks (hypothesis) of the oracle's operators on random
shapes and values: L and L^T are adjoint (Eqs. 5-6 and their Frobenius
adjoint), and P_C (Eq. 26, with a support mask) and P_S (Eqs. 20, 33, 35, 37)
are projections: idempotent, into their sets (membership written here from
Eqs. 17, 25, 32, 34, 36), nonexpansive, and satisfying the variational
inequality <g - P g, z - P g> <= 0 for every z in the set."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st
from hypothesis.extra import numpy as hnp

from oracle import tv

SET = settings(max_examples=60, deadline=None)
EPS = 1e-12
vals = st.floats(-3.0, 3.0, allow_nan=False, allow_infinity=False, width=64)


def planes(m, n):
    return hnp.arrays(np.float64, (m, n), elements=vals)


@st.composite
def image_pair(draw, lo=1, hi=7):
    m, n = draw(st.integers(lo, hi)), draw(st.integers(lo, hi))
    return draw(planes(m, n)), draw(planes(m, n))


@st.composite
def dual_case(draw):
    m, n = draw(st.integers(2, 6)), draw(st.integers(2, 6))

    def q():
        return (draw(planes(m - 1, n)), draw(planes(m, n - 1)), draw(planes(m - 1, n)), draw(planes(m, n - 1)))
    return (m, n), q(), q(), q()


def inner(a, b):
    return float(sum(np.sum(x * y) for x, y in zip(a, b)))


def sub(a, b):
    return tuple(x - y for x, y in zip(a, b))


def norm(a):
    return np.sqrt(inner(a, a))


def in_S(q, kind, alpha):
    """Membership in S, written from the set definitions: interior groups are
    (j, k) with j < m-1, k < n-1; Q1 = (r1, s1) lives on (m-1) x n, Q2 =
    (r2, s2) on m x (n-1)."""
    r1, r2, s1, s2 = q
    a, b = alpha, 1.0 - alpha
    tol = 1e-12
    if kind == "1i":
        inner4 = r1[:, :-1] ** 2 + r2[:-1, :] ** 2 + s1[:, :-1] ** 2 + s2[:-1, :] ** 2
        return (np.all(inner4 <= 1 + tol) and np.all(r1[:, -1] ** 2 + s1[:, -1] ** 2 <= 1 + tol)
                and np.all(r2[-1, :] ** 2 + s2[-1, :] ** 2 <= 1 + tol))
    if kind == "1a":
        return np.all(r1 ** 2 + s1 ** 2 <= 1 + tol) and np.all(r2 ** 2 + s2 ** 2 <= 1 + tol)
    if kind == "2i":
        return (np.all(r1[:, :-1] ** 2 + r2[:-1, :] ** 2 <= a * a + tol)
                and np.all(s1[:, :-1] ** 2 + s2[:-1, :] ** 2 <= b * b + tol)
                and np.all(np.abs(r1[:, -1]) <= a + tol) and np.all(np.abs(r2[-1, :]) <= a + tol)
                and np.all(np.abs(s1[:, -1]) <= b + tol) and np.all(np.abs(s2[-1, :]) <= b + tol))
    return (np.all(np.abs(r1) <= a + tol) and np.all(np.abs(r2) <= a + tol)
            and np.all(np.abs(s1) <= b + tol) and np.all(np.abs(s2) <= b + tol))


@SET
@given(image_pair(), st.data())
def test_L_and_LT_are_adjoint(uv, data):
    u, _ = uv
    m, n = u.shape
    a1 = data.draw(planes(m - 1, n))
    a2 = data.draw(planes(m, n - 1))
    d1, d2 = tv.L(u)
    lhs = float(np.sum(d1 * a1) + np.sum(d2 * a2))
    rhs = float(np.sum(u * tv.LT(a1, a2, (m, n))))
    assert abs(lhs - rhs) <= 1e-10 * (1.0 + abs(lhs))


@SET
@given(image_pair(), image_pair(), st.sampled_from(["modulus", "none"]), st.booleans(), st.data())
def test_P_C_is_a_projection(g, z0, constraint, use_mask, data):
    m, n = g[0].shape
    mask = data.draw(hnp.arrays(np.uint8, (m, n), elements=st.integers(0, 1))) if use_mask else None
    other = (data.draw(planes(m, n)), data.draw(planes(m, n)))
    z = tv.P_C(*[np.resize(a, (m, n)) for a in z0], constraint, mask)
    p = tv.P_C(*g, constraint, mask)
    # idempotent and in C
    pp = tv.P_C(*p, constraint, mask)
    assert np.allclose(pp[0], p[0], atol=EPS) and np.allclose(pp[1], p[1], atol=EPS)
    if constraint == "modulus":
        assert np.all(p[0] ** 2 + p[1] ** 2 <= 1 + 1e-12)
    if mask is not None:
        assert np.all(p[0][mask == 0] == 0) and np.all(p[1][mask == 0] == 0)
    # nonexpansive
    po = tv.P_C(*other, constraint, mask)
    assert norm(sub(p, po)) <= norm(sub(g, other)) + 1e-12
    # variational inequality against a point of C
    assert inner(sub(g, p), sub(z, p)) <= 1e-10


@SET
@given(dual_case(), st.sampled_from(["1i", "1a", "2i", "2a"]), st.floats(0.0, 1.0))
def test_P_S_is_a_projection(case, kind, alpha):
    _, g, other, z0 = case
    p = tv.P_S(g, kind, alpha)
    assert in_S(p, kind, alpha)
    pp = tv.P_S(p, kind, alpha)
    assert all(np.allclose(a, b, atol=1e-12) for a, b in zip(pp, p))
    po = tv.P_S(other, kind, alpha)
    assert norm(sub(p, po)) <= norm(sub(g, other)) + 1e-12
    z = tv.P_S(z0, kind, alpha)
    assert in_S(z, kind, alpha)
    assert inner(sub(g, p), sub(z, p)) <= 1e-10
