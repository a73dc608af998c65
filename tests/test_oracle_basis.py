"""Pins for the oracle's quadrature and orthonormal basis (Section 2, eqs.
triangleDomain, triangleBasis, massMatrix2D)."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import basis, quadrature


def _exact_monomial_integral(a, b):
    """int_I r^a s^b dr ds in exact rational arithmetic: with r = 2 xi - 1,
    s = 2 eta - 1 over the unit right triangle, int xi^p eta^q = p! q!/(p+q+2)!."""
    tot = Fraction(0)
    for p in range(a + 1):
        for q in range(b + 1):
            c = (math.comb(a, p) * (2 ** p) * (-1) ** (a - p) * math.comb(b, q) * (2 ** q) * (-1) ** (b - q))
            tot += c * Fraction(math.factorial(p) * math.factorial(q), math.factorial(p + q + 2))
    return 4 * tot


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_triangle_rule_exact_to_degree(n):
    r, s, w = quadrature.triangle_rule(n)
    for a in range(2 * n):
        for b in range(2 * n - a):
            got = np.sum(w * r ** a * s ** b)
            assert abs(got - float(_exact_monomial_integral(a, b))) < 1e-13


def test_triangle_rule_not_exact_beyond_degree():
    # the collapsed 2x2 rule is exact to degree 3 only: degree 4 must miss
    r, s, w = quadrature.triangle_rule(2)
    assert abs(np.sum(w * s ** 4) - float(_exact_monomial_integral(0, 4))) > 1e-6


@pytest.mark.parametrize("N", [1, 2, 3])
def test_edge_rule(N):
    t, w = quadrature.edge_rule(N)
    n = len(t)
    assert np.allclose(t, -t[::-1], atol=0, rtol=0)
    for k in range(2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * t ** k) - exact) < 1e-14
    assert 2 * n - 1 >= 3 * N


@pytest.mark.parametrize("N", [1, 2, 3])
def test_orthonormal_on_reference(N):
    r, s, w = quadrature.triangle_rule(N + 2)
    V = basis.vandermonde(N, r, s)
    G = np.einsum("q,qi,qj->ij", w, V, V)
    assert np.allclose(G, np.eye(basis.n_modes(N)), atol=1e-14)


def test_mode_ordering_is_the_printed_index():
    # m = j + (N+1) i + 1 - i(i-1)/2 (1-based) enumerates 1..Np without gaps
    for N in (1, 2, 3):
        ml = basis.mode_list(N)
        assert [n for n, _, _ in ml] == list(range(basis.n_modes(N)))
    assert [(i, j) for _, i, j in basis.mode_list(2)] == [(0, 0), (0, 1), (0, 2), (1, 0), (1, 1), (2, 0)]


def test_p1_closed_forms():
    """N = 1 basis written out by hand from the Jacobi definitions:
    P_0 = 1/sqrt2, P_0^{(1,0)} = 1/sqrt2, P_1^{(1,0)}(s) = (3s+1)/2 (unit
    norm with weight 1-s), P_1(a) = sqrt(3/2) a, P_0^{(3,0)} = 1/2, so
    psi_0 = 1/sqrt2, psi_1 = (3s+1)/2, psi_2 = sqrt3 (1 + 2r + s)/2."""
    rng = np.random.default_rng(0)
    xi = rng.uniform(size=(50, 2))
    xi = np.where(xi.sum(1, keepdims=True) > 1, 1 - xi, xi)
    r, s = 2 * xi[:, 0] - 1, 2 * xi[:, 1] - 1
    V = basis.vandermonde(1, r, s)
    assert np.allclose(V[:, 0], 1 / math.sqrt(2), atol=1e-15)
    assert np.allclose(V[:, 1], (3 * s + 1) / 2, atol=1e-14)
    assert np.allclose(V[:, 2], math.sqrt(3) * (1 + 2 * r + s) / 2, atol=1e-14)


@pytest.mark.parametrize("N", [1, 2, 3])
def test_gradients_match_finite_differences(N):
    rng = np.random.default_rng(N)
    xi = rng.uniform(0.05, 0.45, size=(40, 2))
    r, s = 2 * xi[:, 0] - 1, 2 * xi[:, 1] - 1
    Dr, Ds = basis.grad_vandermonde(N, r, s)
    h = 1e-6
    fr = (basis.vandermonde(N, r + h, s) - basis.vandermonde(N, r - h, s)) / (2 * h)
    fs = (basis.vandermonde(N, r, s + h) - basis.vandermonde(N, r, s - h)) / (2 * h)
    assert np.allclose(Dr, fr, atol=2e-8)
    assert np.allclose(Ds, fs, atol=2e-8)


def test_physical_rule_area_and_exactness():
    P = np.array([[[0.0, 0.0], [2.0, 0.0], [0.0, 1.0]]])
    x, y, w = quadrature.physical_rule_on_triangle(P, 3)
    assert abs(w.sum() - 1.0) < 1e-15
    # int over that triangle of x^2 y = 2*1 * int_T (2u)^2 v = 8 * 2!1!/5! = 2/15
    assert abs(np.sum(w * x ** 2 * y) - 2.0 / 15.0) < 1e-15
