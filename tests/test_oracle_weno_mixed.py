"""Pins of the mixed WENO oracle (oracle/weno_mixed.py) on the CSWENO
subcell stencils, N = 2: the big stencil's quadratic reproduces quadratic
data and the linear weights give it back for any data, linear data with
the nonlinear weights, the smoothness indicator of p_0 and the weights of
one cell against scalar arithmetic (edge-midpoint quadrature, explicit
derivatives), the weights next to a jump, and the order on smooth data."""
import math

import numpy as np
import pytest

from oracle import weno_mixed as wm
from oracle.dg import DG
from oracle.mesh import BC_PERIODIC, BC_TRANSMISSIVE, INFO_BOUNDARY, Mesh
from paper_2106_06280_amd import inputs


def _case(n=7, eq=0, seed=11):
    v, t = inputs.jittered_mesh(n, seed=seed)
    M = Mesh(v, t, BC_TRANSMISSIVE)
    d = DG(M, 2, eq)
    E = np.nonzero(~np.any((M.info & (INFO_BOUNDARY | 0x3C)) != 0, axis=1))[0]
    return M, d, E


def test_quadratic_data_reproduced_with_the_linear_weights():
    """omega = gamma: gamma_0 p_0 + sum_j gamma_j L_j = Q, and Q is exact on
    quadratic data, so the reconstruction returns the data's own
    coefficients (against the DG projection of the quadratic); a cubic term
    is not reproduced."""
    M, d, E = _case()
    U = d.project(lambda x, y: 0.4 + 0.7 * x - 0.5 * y + 0.9 * x * x - 0.4 * x * y + 0.3 * y * y)
    out = wm.reconstruct_mixed(d, U, E, linear_only=True)
    assert np.abs(out - U[E]).max() < 1e-12
    Uc = d.project(lambda x, y: 0.4 + 0.7 * x + 1.5 * x ** 3)
    assert np.abs(wm.reconstruct_mixed(d, Uc, E, linear_only=True) - Uc[E]).max() > 1e-6


def test_linear_weights_give_back_the_big_stencil_fit():
    """For rough data too: with omega = gamma the combined coefficients are
    Q's (the positive-weight identity of the mixed form)."""
    M, d, E = _case()
    U = d.project(lambda x, y: 0.4 + np.sin(5 * x) * np.cos(3 * y) + np.where(x + y > 1.1, 0.6, 0.0))
    _, info = wm.reconstruct_mixed(d, U, E, linear_only=True, return_info=True)
    assert np.abs(info["cR"] - info["cQ"]).max() < 1e-13 * max(1.0, np.abs(info["cQ"]).max())
    assert wm.GAMMA0 > 0 and wm.GAMMA_SMALL > 0 and abs(wm.GAMMA0 + 6 * wm.GAMMA_SMALL - 1.0) < 1e-15


@pytest.mark.parametrize("eq", [0, 1])
def test_linear_data_reproduced_by_the_nonlinear_weights(eq):
    """Linear data: Q, every L_j and hence p_0 are the data, so any
    normalised weights return it."""
    M, d, E = _case(eq=eq)
    if eq == 0:
        U = d.project(lambda x, y: 0.4 + 0.7 * x - 0.5 * y)
    else:
        U = d.project(lambda x, y: np.stack([1.0 + 0.2 * x - 0.1 * y, 0.3 + 0.1 * x, -0.2 + 0.05 * y,
                                             2.5 + 0.1 * x + 0.2 * y], -1))
    assert np.abs(wm.reconstruct_mixed(d, U, E) - U[E]).max() < 1e-12


def _beta_scalar(V, x0, y0, h0, c):
    """sum over |alpha| = 1, 2 of |D0|^{|alpha|-1} int (D^alpha p)^2 for
    p = c1 xi + c2 eta + c3 xi^2 + c4 xi eta + c5 eta^2 (+ const), xi =
    (x - x0)/h0: the first derivatives are linear, their squares integrate
    exactly by the edge-midpoint rule; the second derivatives are
    constants."""
    P = [np.array(V[i], float) for i in range(3)]
    area = 0.5 * abs((P[1][0] - P[0][0]) * (P[2][1] - P[0][1]) - (P[2][0] - P[0][0]) * (P[1][1] - P[0][1]))
    first = 0.0
    for i in range(3):
        m = 0.5 * (P[i] + P[(i + 1) % 3])
        xi, eta = (m[0] - x0) / h0, (m[1] - y0) / h0
        px = (c[0] + 2 * c[2] * xi + c[3] * eta) / h0
        py = (c[1] + c[3] * xi + 2 * c[4] * eta) / h0
        first += area / 3.0 * (px * px + py * py)
    pxx, pxy, pyy = 2 * c[2] / h0 ** 2, c[3] / h0 ** 2, 2 * c[4] / h0 ** 2
    return first + area * area * (pxx * pxx + pxy * pxy + pyy * pyy)


def test_weights_and_reconstruction_of_one_cell_in_scalar_arithmetic():
    """One element, one field, rough data: p_0 from Q and the L_j with the
    stated linear weights, beta_0 by _beta_scalar, beta_j = |D0| |c_j|^2 /
    h0^2, the classical weights, and R's moments by the degree-4 rule,
    against the oracle's."""
    from oracle import basis
    M, d, E = _case()
    U = d.project(lambda x, y: 0.4 + np.sin(3 * x) * np.cos(2 * y) + np.where(x > 0.55, 0.5, 0.0))
    e = E[len(E) // 2]
    out, info = wm.reconstruct_mixed(d, U, [e], return_info=True)
    cQ = info["cQ"][0, :, 0]
    cL = [c[0, :, 0] for c in info["cL"]]
    c0 = cQ.copy()
    for c in cL:
        c0[:2] -= 0.025 * c
    c0 /= 0.85
    assert np.allclose(c0, info["c0"][0, :, 0], rtol=1e-13, atol=1e-15)
    V, x0, y0, h0 = M.V[e], info["x0"][0], info["y0"][0], info["h0"][0]
    area = info["area0"][0]
    b = [_beta_scalar(V, x0, y0, h0, c0)] + [area * (c @ c) / h0 ** 2 for c in cL]
    assert np.allclose(b, [x[0, 0] for x in info["beta"]], rtol=1e-12, atol=0.0)
    g = np.array([0.85] + [0.025] * 6)
    om = g / (1e-6 + np.array(b)) ** 2
    om /= om.sum()
    assert np.allclose(om, info["omega"][0, :, 0], rtol=1e-12)
    cR = om[0] * c0
    for j, c in enumerate(cL):
        cR[:2] += om[j + 1] * c
    r, s, w = info["rule"]
    Rq = info["fbar0"][0, 0] + info["phi"][0] @ cR
    mom = np.einsum("q,q,qi->i", w, Rq, basis.vandermonde(2, r, s))
    assert np.allclose(mom[1:], out[0, 0, 1:], rtol=1e-12, atol=1e-14)


def test_stencils_across_a_jump_lose_their_weight():
    """A jump that crosses only the neighbour across face 0 of a cell: the
    small stencils without that neighbour (single neighbours 1 and 2, the
    sector of faces 1 and 2) take almost all the weight, p_0 and the
    stencils with it almost none."""
    M, d, E = _case(n=9)
    for e in E:
        nb0 = M.nbr[e, 0]
        c_nb = M.V[nb0].mean(axis=0)
        c_e = M.V[e].mean(axis=0)
        n = c_nb - c_e
        n /= np.linalg.norm(n)
        # a line between the cell and that neighbour's far side, parallel to face 0
        off = n @ (0.5 * (M.V[e, 0] + M.V[e, 1])) + 0.6 * (n @ (c_nb - 0.5 * (M.V[e, 0] + M.V[e, 1])))
        U = d.project(lambda x, y: np.where(n[0] * x + n[1] * y > off, 1.0, 0.0))
        cells_hit = [k for k in range(M.K) if np.ptp(U[k, 0]) > 0 or abs(U[k, 0, 1:]).max() > 1e-12]
        if nb0 not in cells_hit or set(cells_hit) & {e, M.nbr[e, 1], M.nbr[e, 2]}:
            continue  # the jump must touch neighbour 0 only
        _, info = wm.reconstruct_mixed(d, U, [e], return_info=True)
        om = info["omega"][0, :, 0]
        away = om[[2, 3, 5]].sum()  # L for faces 1, 2 and the sector (1, 2)
        assert away > 0.99, om
        return
    pytest.skip("no cell with a jump across its neighbour 0 only on this mesh")


def test_single_application_order_on_smooth_data():
    """Every cell limited once on smooth Burgers data: the error falls at
    the design order 3 within 0.35."""
    ic = inputs.BurgersSine()
    errs = []
    for n in (16, 32, 64):
        v, t = inputs.jittered_mesh(n, -2, 2, -2, 2, seed=7)
        M = Mesh(v, t, BC_PERIODIC, (4.0, 4.0))
        d = DG(M, 2, 0)
        U = d.project(ic)
        errs.append(d.errors(wm.limit_mixed(d, U, np.ones(M.K, bool)), ic)[0])
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert orders[-1] > 2.65, (errs, orders)


def test_rejects_other_degrees():
    v, t = inputs.jittered_mesh(3, seed=1)
    d = DG(Mesh(v, t, BC_TRANSMISSIVE), 1, 0)
    with pytest.raises(ValueError):
        wm.reconstruct_mixed(d, d.project(lambda x, y: x), [0])
