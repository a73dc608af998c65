"""Quadrature rules on the reference triangle and on the reference edge.

The paper does not name its volume or edge quadratures (Section 2 only
says the weak form is integrated).  Reading used here:

* volume: collapsed-coordinate (Duffy) rule, Gauss-Legendre in a times
  Gauss-Jacobi(1,0) in b, n points per direction, exact for total degree
  2n-1 on I = {(r,s): r,s >= -1, r+s <= 0} (Section 2, eq. triangleDomain);
  the residual uses n_v = ceil(3N/2);
* edge: Gauss-Legendre with n_e = ceil((3N+1)/2) points on [-1, 1].

Nodes come from scipy's Gauss routines (a library primitive).  Pinned by
tests/test_oracle_basis.py against closed-form monomial integrals.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import roots_jacobi, roots_legendre


def gauss_legendre(n: int):
    x, w = roots_legendre(n)
    return np.asarray(x, dtype=np.float64), np.asarray(w, dtype=np.float64)


def gauss_jacobi(n: int, alpha: float, beta: float = 0.0):
    x, w = roots_jacobi(n, alpha, beta)
    return np.asarray(x, dtype=np.float64), np.asarray(w, dtype=np.float64)


def triangle_rule(n: int):
    """Collapsed rule on I.  Returns r, s, w with sum(w) = |I| = 2."""
    a, wa = gauss_legendre(n)
    b, wb = gauss_jacobi(n, 1.0, 0.0)
    A, B = np.meshgrid(a, b, indexing="ij")
    r = 0.5 * (1.0 + A) * (1.0 - B) - 1.0
    s = B
    # dr ds = (1-b)/2 da db; the factor (1-b) is the Jacobi weight.
    w = 0.5 * wa[:, None] * wb[None, :]
    return r.ravel(), s.ravel(), w.ravel()


def triangle_rule_for_degree(d: int):
    return triangle_rule(max(1, (d + 2) // 2))


def volume_points(N: int) -> int:
    return int(math.ceil(3 * N / 2))


def edge_points(N: int) -> int:
    return int(math.ceil((3 * N + 1) / 2))


def edge_rule(N: int):
    t, w = gauss_legendre(edge_points(N))
    # enforce exact mirror symmetry t[g] = -t[n-1-g] so that both sides of an
    # edge see the same physical points
    t = 0.5 * (t - t[::-1])
    w = 0.5 * (w + w[::-1])
    return t, w


def face_reference_points(f: int, t):
    """Reference coordinates of edge parameter t in [-1,1] on local face f.

    Face f runs from vertex f to vertex f+1 (mod 3); reference vertices are
    (-1,-1), (1,-1), (-1,1)."""
    t = np.asarray(t, dtype=np.float64)
    if f == 0:
        return t, -np.ones_like(t)
    if f == 1:
        return -t, t
    if f == 2:
        return -np.ones_like(t), -t
    raise ValueError(f)


def physical_rule_on_triangle(P, n: int):
    """Map the collapsed rule to physical triangles P [..., 3, 2].

    Returns x [..., q], y [..., q], w [..., q] with sum(w) = area."""
    r, s, w = triangle_rule(n)
    P = np.asarray(P, dtype=np.float64)
    p0 = P[..., 0, :]
    p1 = P[..., 1, :]
    p2 = P[..., 2, :]
    lam1 = 0.5 * (1.0 + r)
    lam2 = 0.5 * (1.0 + s)
    x = p0[..., 0, None] + lam1 * (p1[..., 0, None] - p0[..., 0, None]) + lam2 * (p2[..., 0, None] - p0[..., 0, None])
    y = p0[..., 1, None] + lam1 * (p1[..., 1, None] - p0[..., 1, None]) + lam2 * (p2[..., 1, None] - p0[..., 1, None])
    area2 = (p1[..., 0] - p0[..., 0]) * (p2[..., 1] - p0[..., 1]) - (p2[..., 0] - p0[..., 0]) * (p1[..., 1] - p0[..., 1])
    J = 0.25 * np.abs(area2)  # |area|/2: reference area is 2
    return x, y, J[..., None] * w
