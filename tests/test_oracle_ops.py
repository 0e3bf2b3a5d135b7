"""Pins for the oracle's linear operators, TV definitions and projections.

Each check compares against something other than the oracle's own formula: a
dense matrix built entry by entry, the adjoint identity, loop-form sums,
support-function identities, or the defining properties of a Euclidean
projection.
"""
import numpy as np
import pytest

from oracle import pdhg, tv

SHAPES = [(1, 1), (1, 6), (5, 1), (2, 2), (4, 4), (3, 5), (7, 4)]


def rand_dual(m, n, rng, scale=1.0):
    return (rng.standard_normal((m - 1, n)) * scale, rng.standard_normal((m, n - 1)) * scale,
            rng.standard_normal((m - 1, n)) * scale, rng.standard_normal((m, n - 1)) * scale)


def flat(q):
    return np.concatenate([np.ravel(a) for a in q])


@pytest.mark.parametrize("shape", SHAPES)
def test_L_matches_dense_difference_matrix(shape, rng):
    m, n = shape
    D, _ = pdhg.difference_matrix(m, n)
    x = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    p = flat(tv.L_pair(x.real, x.imag))
    np.testing.assert_allclose(p, D @ pdhg.to_vec(x), atol=1e-14)


@pytest.mark.parametrize("shape", SHAPES)
def test_LT_is_adjoint(shape, rng):
    m, n = shape
    x = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    q = rand_dual(m, n, rng)
    lhs = float(flat(tv.L_pair(x.real, x.imag)) @ flat(q))
    lu, lv = tv.LT_pair(q, (m, n))
    rhs = float(np.sum(x.real * lu) + np.sum(x.imag * lv))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
    # and against the transpose of the dense matrix
    D, _ = pdhg.difference_matrix(m, n)
    np.testing.assert_allclose(np.concatenate([lu.ravel(), lv.ravel()]), D.T @ flat(q), atol=1e-13)


def test_L_kills_constants_and_LT_sums_to_zero(rng):
    c = np.full((5, 6), 0.3 - 0.7j)
    for d in tv.L_pair(c.real, c.imag):
        assert np.all(d == 0)
    q = rand_dual(5, 6, rng)
    lu, lv = tv.LT_pair(q, (5, 6))
    assert abs(lu.sum()) < 1e-12 and abs(lv.sum()) < 1e-12


def test_operator_norm_bound_gives_16_lambda_squared():
    """||L||^2 <= 8 (so grad h has Lipschitz constant 2 lam^2 * 8 = 16 lam^2,
    the paper's printed bound) and the bound is approached on a large grid."""
    import json, os
    const = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
    assert const["lipschitz_factor"]["value"] == 2 * 8
    for (m, n) in [(3, 4), (64, 64)]:
        rng = np.random.default_rng(0)
        u = rng.standard_normal((m, n))
        est = 0.0
        for _ in range(400):
            a1, a2 = tv.L(u)
            v = tv.LT(a1, a2, (m, n))
            est = np.linalg.norm(v) / np.linalg.norm(u)
            u = v / np.linalg.norm(v)
        assert est <= 8.0 + 1e-9
        if m == 64:
            assert est > 7.9
    D, _ = pdhg.difference_matrix(4, 4)
    assert np.linalg.norm(D, 2) ** 2 <= 8.0


@pytest.mark.parametrize("shape", [(1, 1), (1, 5), (4, 1), (3, 3), (5, 4)])
def test_tv_vectorised_equals_loop(shape, rng):
    u = rng.standard_normal(shape)
    for iso in (True, False):
        assert abs(tv.tv_vec(u, iso) - tv.tv_real(u, iso)) < 1e-12


@pytest.mark.parametrize("kind", tv.KINDS)
@pytest.mark.parametrize("shape", [(1, 4), (4, 1), (3, 5), (4, 4)])
def test_tv_matches_dense_group_form(kind, shape, rng):
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    alpha = 0.3
    prob = pdhg.Problem(np.zeros(shape), 1.0, kind, alpha)
    assert abs(tv.tv(x, kind, alpha) - prob.tv(pdhg.to_vec(x))) < 1e-12


def test_tv_real_reductions(rng):
    u = rng.standard_normal((5, 6))
    # type-I of a real image is the real TV (Eqs. 3-4 vs 7-8)
    assert abs(tv.tv(u + 0j, "1i") - tv.tv_real(u, True)) < 1e-12
    assert abs(tv.tv(u + 0j, "1a") - tv.tv_real(u, False)) < 1e-12
    v = rng.standard_normal((5, 6))
    assert abs(tv.tv(u + 1j * v, "2i", 0.3) - (0.3 * tv.tv_real(u, True) + 0.7 * tv.tv_real(v, True))) < 1e-12
    assert abs(tv.tv(u + 1j * v, "2a", 0.3) - (0.3 * tv.tv_real(u, False) + 0.7 * tv.tv_real(v, False))) < 1e-12


@pytest.mark.parametrize("kind", tv.KINDS)
@pytest.mark.parametrize("shape", [(1, 5), (5, 1), (4, 4), (3, 6)])
def test_support_function_identity(kind, shape, rng):
    """TV(x) = max_{q in S} <q, L x>: every q in S gives <= TV(x), and the
    group-normalised L x (P_S of a huge multiple of L x) attains it. This ties
    the sets S (Eqs. 17, 32, 34, 36) and projections (20, 33, 35, 37) to the
    TV definitions (7)-(10)."""
    alpha = 0.35
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    p = tv.L_pair(x.real, x.imag)
    T = tv.tv(x, kind, alpha)
    qstar = tv.P_S(tuple(1e9 * a for a in p), kind, alpha)
    assert abs(float(flat(qstar) @ flat(p)) - T) < 1e-8 * max(1, T)
    for _ in range(5):
        q = tv.P_S(rand_dual(*shape, rng, 2.0), kind, alpha)
        assert float(flat(q) @ flat(p)) <= T + 1e-12


# ----------------------------------------------------------------------------
# projections
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("constraint", tv.CONSTRAINTS)
def test_PC_projection_properties(constraint, rng):
    m, n = 6, 5
    w = (rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))) * 1.5
    mask = (rng.random((m, n)) > 0.3).astype(np.uint8)
    for mk in (None, mask):
        yu, yv = tv.P_C(w.real, w.imag, constraint, mk)
        y = yu + 1j * yv
        if constraint == "modulus":
            assert np.all(np.abs(y) <= 1 + 1e-15)
        if mk is not None:
            assert np.all(y[mk == 0] == 0)
        # idempotent; a pixel the first pass scaled to modulus 1 can come out one
        # rounding above 1 in float64, and the second pass then rescales it by 1 - 2^-52
        y2u, y2v = tv.P_C(yu, yv, constraint, mk)
        np.testing.assert_allclose(y2u, yu, rtol=4e-16, atol=0)
        np.testing.assert_allclose(y2v, yv, rtol=4e-16, atol=0)
        # variational inequality <w - Pw, z - Pw> <= 0 for z in C
        for _ in range(5):
            z = (rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n)))
            zu, zv = tv.P_C(z.real, z.imag, constraint, mk)
            val = np.sum((w.real - yu) * (zu - yu) + (w.imag - yv) * (zv - yv))
            assert val <= 1e-12


def test_PC_pixel_brute_force(rng):
    """Per pixel, P_C minimises |z - w| over the closed unit disc: compare with a
    dense angular/radial grid search."""
    th = np.linspace(-np.pi, np.pi, 2001)
    rr = np.linspace(0, 1, 401)
    Z = (rr[:, None] * np.exp(1j * th[None, :])).ravel()
    for _ in range(10):
        w = complex(*(rng.standard_normal(2) * 1.3))
        yu, yv = tv.P_C(np.array([[w.real]]), np.array([[w.imag]]))
        best = Z[np.argmin(np.abs(Z - w))]
        assert abs((yu[0, 0] + 1j * yv[0, 0]) - best) < 5e-3


@pytest.mark.parametrize("kind", tv.KINDS)
@pytest.mark.parametrize("alpha", [0.5, 0.2, 0.0, 1.0])
def test_PS_projection_properties(kind, alpha, rng):
    m, n = 5, 4
    g = rand_dual(m, n, rng, 1.5)
    p = tv.P_S(g, kind, alpha)
    prob = pdhg.Problem(np.zeros((m, n)), 1.0, kind, alpha)
    assert prob.in_dual_set(flat(p))
    p2 = tv.P_S(p, kind, alpha)
    np.testing.assert_allclose(flat(p2), flat(p), atol=1e-15)
    for _ in range(5):
        z = tv.P_S(rand_dual(m, n, rng, 1.5), kind, alpha)
        # variational inequality characterises the Euclidean projection
        assert float((flat(g) - flat(p)) @ (flat(z) - flat(p))) <= 1e-12
        # nonexpansive
        h = rand_dual(m, n, rng, 1.5)
        ph = tv.P_S(h, kind, alpha)
        assert np.linalg.norm(flat(p) - flat(ph)) <= np.linalg.norm(flat(g) - flat(h)) + 1e-12


@pytest.mark.parametrize("kind", tv.KINDS)
def test_PS_matches_dense_group_projection(kind, rng):
    m, n = 4, 5
    alpha = 0.4
    g = rand_dual(m, n, rng, 1.5)
    prob = pdhg.Problem(np.zeros((m, n)), 1.0, kind, alpha)
    np.testing.assert_allclose(flat(tv.P_S(g, kind, alpha)), prob.proj_dual(flat(g)), atol=1e-14)
