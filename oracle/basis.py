"""Orthonormal modal basis on the reference triangle (Section 2, eqs.
triangleDomain and triangleBasis).

psi_m(r,s) = sqrt(2) P_i(a) P_j^{(2i+1,0)}(b) (1-b)^i with
a = 2(1+r)/(1-s) - 1, b = s, and the 1-based index
m = j + (N+1) i + 1 - i(i-1)/2 over i, j >= 0, i + j <= N.
The Jacobi polynomials are taken L2-normalised on [-1, 1] with their
weights, which makes the basis orthonormal on I (the paper calls it
orthonormal).  The oracle uses the 0-based index n = m - 1.

Jacobi values come from scipy.special.eval_jacobi (a library primitive).
Pinned by tests/test_oracle_basis.py: orthonormality, the closed forms of
the N = 1 functions derived by hand from the definition, and
finite-difference gradients.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import eval_jacobi


def n_modes(N: int) -> int:
    return (N + 1) * (N + 2) // 2


def mode_list(N: int):
    """[(n, i, j)] in the paper's ordering, n 0-based."""
    out = []
    for i in range(N + 1):
        for j in range(N + 1 - i):
            m = j + (N + 1) * i + 1 - (i * (i - 1)) // 2
            out.append((m - 1, i, j))
    out.sort()
    assert [t[0] for t in out] == list(range(n_modes(N)))
    return out


def jacobi_normalised(x, n: int, alpha: float):
    """P_n^{(alpha,0)} scaled to unit norm with weight (1-x)^alpha."""
    norm2 = 2.0 ** (alpha + 1.0) / (2 * n + alpha + 1.0)
    return eval_jacobi(n, alpha, 0.0, x) / math.sqrt(norm2)


def jacobi_normalised_deriv(x, n: int, alpha: float):
    """d/dx of jacobi_normalised: (n+alpha+1)/2 P_{n-1}^{(alpha+1,1)}."""
    if n == 0:
        return np.zeros_like(np.asarray(x, dtype=np.float64))
    norm2 = 2.0 ** (alpha + 1.0) / (2 * n + alpha + 1.0)
    return 0.5 * (n + alpha + 1.0) * eval_jacobi(n - 1, alpha + 1.0, 1.0, x) / math.sqrt(norm2)


def _collapse(r, s):
    r = np.asarray(r, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    denom = 1.0 - s
    safe = np.abs(denom) > 1e-14
    a = np.where(safe, 2.0 * (1.0 + r) / np.where(safe, denom, 1.0) - 1.0, -1.0)
    return a, s


def vandermonde(N: int, r, s):
    """psi_n(r_q, s_q) as an array [..., q, Np]."""
    a, b = _collapse(r, s)
    cols = []
    for n, i, j in mode_list(N):
        cols.append(math.sqrt(2.0) * jacobi_normalised(a, i, 0.0)
                    * jacobi_normalised(b, j, 2 * i + 1.0) * (1.0 - b) ** i)
    return np.stack(cols, axis=-1)


def grad_vandermonde(N: int, r, s):
    """(d psi_n/dr, d psi_n/ds) at (r_q, s_q), each [..., q, Np]."""
    a, b = _collapse(r, s)
    dr, ds = [], []
    for n, i, j in mode_list(N):
        A = jacobi_normalised(a, i, 0.0)
        dA = jacobi_normalised_deriv(a, i, 0.0)
        B = jacobi_normalised(b, j, 2 * i + 1.0)
        dB = jacobi_normalised_deriv(b, j, 2 * i + 1.0)
        om = 1.0 - b
        # da/dr = 2/(1-s); da/ds = (1+a)/(1-s)
        if i == 0:
            d_r = np.zeros_like(a)
            d_s = math.sqrt(2.0) * A * dB
        else:
            d_r = math.sqrt(2.0) * dA * B * 2.0 * om ** (i - 1)
            d_s = math.sqrt(2.0) * (dA * (1.0 + a) * B * om ** (i - 1)
                                    + A * (dB * om ** i - i * B * om ** (i - 1)))
        dr.append(d_r)
        ds.append(d_s)
    return np.stack(dr, axis=-1), np.stack(ds, axis=-1)
