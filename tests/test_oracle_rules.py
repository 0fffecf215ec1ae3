"""Pins for the oracle's reference data: quadrature exactness against closed
forms, orthonormality of the Koornwinder basis, interpolation nodes."""

import math

import numpy as np
import pytest

from oracle import rules


def simplex_monomial(a, b):
    """int_T x^a y^b dA = a! b! / (a + b + 2)!."""
    return math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)


@pytest.mark.parametrize("q", [2, 3, 4, 7, 8, 12, 16, 20])
def test_collapsed_gauss_exact_through_2q_minus_1(q):
    X, W = rules.collapsed_gauss(q)
    assert X.shape == (q * q, 2)
    assert abs(W.sum() - 0.5) < 1e-15
    for a in range(2 * q):
        for b in range(2 * q - a):
            got = np.sum(W * X[:, 0] ** a * X[:, 1] ** b)
            ref = simplex_monomial(a, b)
            assert abs(got - ref) <= 5e-14 * ref + 1e-17, (a, b)
    # not exact at total degree 2q for every monomial
    errs = [abs(np.sum(W * X[:, 0] ** a * X[:, 1] ** (2 * q - a)) / simplex_monomial(a, 2 * q - a) - 1.0)
            for a in range(2 * q + 1)]
    assert max(errs) > 3e-13
    # nodes strictly inside the simplex
    assert np.all(X[:, 0] > 0) and np.all(X[:, 1] > 0) and np.all(X.sum(1) < 1)


@pytest.mark.parametrize("n", [4, 8, 10, 16])
def test_gauss_legendre01(n):
    x, w = rules.gauss_legendre01(n)
    for k in range(2 * n):
        assert abs(np.sum(w * x ** k) - 1.0 / (k + 1)) < 1e-15


@pytest.mark.parametrize("n", [2, 4, 5, 6, 8])
def test_log_gauss_moments(n):
    """int_0^1 -log(r) r^k dr = 1/(k+1)^2 for k <= 2n - 1."""
    r, w = rules.log_gauss01(n)
    assert np.all((r > 0) & (r < 1)) and np.all(w > 0)
    for k in range(2 * n):
        assert abs(np.sum(w * r ** k) - 1.0 / (k + 1) ** 2) < 2e-16 * 8


@pytest.mark.parametrize("p", [1, 2, 4, 6, 8, 10])
def test_radial_rule_exact_on_r_log_r0r_poly(p):
    """int_0^1 r log(r0 r) r^k dr = log(r0)/(k+2) - 1/(k+2)^2, k <= p."""
    r, alpha, beta = rules.radial_rule(p)
    for r0 in (1e-3, 0.37, 1.0, 4.2):
        for k in range(p + 1):
            got = np.sum((alpha * math.log(r0) + beta) * r ** k)
            ref = math.log(r0) / (k + 2) - 1.0 / (k + 2) ** 2
            assert abs(got - ref) < 1e-15 * (1 + abs(math.log(r0))), (r0, k)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 6, 8, 10])
def test_koornwinder_orthonormal(p):
    X, W = rules.collapsed_gauss(p + 1)
    K = rules.koornwinder(p, X[:, 0], X[:, 1])
    G = K.T @ (W[:, None] * K)
    assert np.abs(G - np.eye(rules.n_basis(p))).max() < 1e-13
    # K_00 is the constant sqrt(2)
    assert np.allclose(K[:, 0], math.sqrt(2.0), atol=1e-15)


@pytest.mark.parametrize("p", [3, 6])
def test_koornwinder_total_degree(p):
    """Column n(n+1)/2 + m has total degree n: orthogonal to every monomial of
    lower degree, and not to some of degree n."""
    X, W = rules.collapsed_gauss(p + 2)
    K = rules.koornwinder(p, X[:, 0], X[:, 1])
    for n in range(p + 1):
        for m in range(n + 1):
            col = K[:, n * (n + 1) // 2 + m]
            for a in range(n):
                for b in range(n - a):
                    assert abs(np.sum(W * col * X[:, 0] ** a * X[:, 1] ** b)) < 1e-13
            hi = max(abs(np.sum(W * col * X[:, 0] ** a * X[:, 1] ** (n - a))) for a in range(n + 1))
            assert hi > 1e-6


def test_koornwinder_collapsed_vertex_limit():
    """At B = (1, 0) every basis function equals its limit along the edge."""
    p = 5
    K_B = rules.koornwinder(p, [1.0], [0.0])[0]
    K_near = rules.koornwinder(p, [1.0 - 1e-9], [0.3e-9])[0]
    assert np.allclose(K_B, K_near, atol=1e-6 * np.abs(K_B).max())


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8, 9, 10])
def test_interp_nodes_and_vandermonde(p):
    X = rules.interp_nodes(p)
    n = rules.n_basis(p)
    assert X.shape == (n, 2)
    assert np.all(X[:, 0] > 0) and np.all(X[:, 1] > 0) and np.all(X.sum(1) < 1)
    # invariant under the symmetry (x, y) -> (y, x) of the simplex
    Xs = np.sort(X[:, 0] + 1e3 * X[:, 1])
    Ys = np.sort(X[:, 1] + 1e3 * X[:, 0])
    assert np.allclose(Xs, Ys, atol=1e-12)
    V = rules.koornwinder(p, X[:, 0], X[:, 1])
    Vi = rules.vandermonde_inverse(p)
    assert np.abs(Vi @ V - np.eye(n)).max() < 1e-12
    assert np.linalg.cond(V) < 100.0
    # interpolation reproduces polynomials of degree p at other points
    rng = np.random.default_rng(p)
    P = rng.dirichlet([1, 1, 1], size=50)[:, 1:]
    for a in range(p + 1):
        for b in range(p + 1 - a):
            vals = X[:, 0] ** a * X[:, 1] ** b
            c = Vi @ vals
            got = rules.koornwinder(p, P[:, 0], P[:, 1]) @ c
            assert np.abs(got - P[:, 0] ** a * P[:, 1] ** b).max() < 1e-12


def test_gll_points():
    """GLL points of order M: end points plus roots of P_M' (checked by the
    exactness of the Lobatto rule they define, degree 2M - 1)."""
    for M in (4, 7, 9):
        x = rules.gauss_lobatto_legendre01(M)
        assert len(x) == M + 1 and x[0] == 0.0 and x[-1] == 1.0
        # Lobatto weights from the Lagrange basis, check exactness
        V = np.vander(x, increasing=True)
        w = np.linalg.solve(V.T, 1.0 / np.arange(1, M + 2))
        for k in range(2 * M):
            assert abs(np.sum(w * x ** k) - 1.0 / (k + 1)) < 1e-12


def test_edge_weights_are_rule_weights():
    for q in (4, 7, 8, 12):
        X, W = rules.collapsed_gauss(q)
        w = rules.edge_weights(q)
        assert w.shape == (3,)
        for e in range(3):
            assert np.any(np.isclose(W, w[e], rtol=0, atol=0))
        # edge CA (x = 0) is nearest to the first row of u-nodes: its q nodes
        assert w[2] == W[:q].max()
