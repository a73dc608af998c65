"""Value pins of the nonlinear-weight chain of the CSWENO limiter (Section 3.2,
Steps 3-4) and of the readings of the fourth member of the N >= 2 hierarchy.

The data are piecewise linear and discontinuous: every element carries its own
linear function u_e(x) = a_e + g_e . (x - c_e).  The average of a linear
function over a subcell is its value at the subcell's centroid, so the linear
function of eq. sigmaEqn's step, p_{1,l}, which vanishes at the centroid of
Delta_l1 and takes ubar_l2 - ubar_l1 and ubar_l3 - ubar_l1 at the other two
centroids, is the neighbour's own linear function minus a constant: its
gradient is g_l, chosen by hand.  So beta_{1,l} = |Delta0| |g_l|^2 (eq.
smoothnessIndicator for a linear function), and sigma_l, beta_1 (eqs.
sigmaEqn, smoothnessIndicatorT1) follow in closed form from the chosen
gradients and the area of Delta0 (computed here from its vertices).  tau
(eqs. tauNonlinearWeightsP1/P2) and omega (eqs. nonLinearWeightsP1/P2) are
then checked with beta_1 from this closed form and beta_2.. of the oracle
(beta of q_l is pinned separately against integrals in closed form).  The
gradients are chosen so that the three beta_{1,l} differ and beta_1, beta_2,
beta_3 differ: a /4 in place of /16 in tau, a dropped outer square in sigma,
or a weight with the wrong linear weight fails these checks.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import csweno
from oracle.dg import DG
from oracle.mesh import BC_PERIODIC, BC_TRANSMISSIVE, INFO_BOUNDARY, Mesh
from paper_2106_06280_amd import inputs

GRADS = [(1.0, 0.0), (0.0, 2.0), (3.0, 1.0)]  # g of the neighbours across faces 0, 1, 2


def _piecewise_linear_case(N, seed=5):
    """A 4 x 4 mesh of [0,4]^2 (element areas near 1/2), an interior cell e0
    and data linear on each element with the hand-chosen gradients GRADS on
    the three neighbours of e0."""
    v, t = inputs.jittered_mesh(4, 0.0, 4.0, 0.0, 4.0, seed=seed)
    M = Mesh(v, t, BC_PERIODIC, (4.0, 4.0))
    interior = np.nonzero(~np.any((M.info & (INFO_BOUNDARY | 0x3C)) != 0, axis=1))[0]
    e0 = int(interior[len(interior) // 2])
    rng = np.random.default_rng(seed)
    K = M.K
    a = 1.0 + 0.5 * rng.standard_normal(K)
    g = 0.7 * rng.standard_normal((K, 2))
    for f in range(3):
        g[M.nbr[e0, f]] = GRADS[f]
    c = M.V.mean(axis=1)  # centroids [K, 2]
    d = DG(M, N, 0)
    U = d.project(lambda x, y: a[:, None] + g[:, 0, None] * (x - c[:, 0, None]) + g[:, 1, None] * (y - c[:, 1, None]))
    return M, d, U, e0, g


def _area(P):
    (x0, y0), (x1, y1), (x2, y2) = P
    return 0.5 * ((x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0))


def _closed_form_beta1(area, grads, eps=1e-10):
    """eqs. sigmaEqn and smoothnessIndicatorT1 for linear functions with the
    given gradients, in exact rational arithmetic on the float inputs."""
    A = Fraction(area)
    b = [A * (Fraction(gx) ** 2 + Fraction(gy) ** 2) for gx, gy in grads]
    inner = ((b[0] - b[1]) ** 2 + (b[1] - b[2]) ** 2 + (b[2] - b[0]) ** 2) / 3
    sig = [Fraction(1, 3) * (1 + inner ** 2 / (bl + Fraction(eps))) for bl in b]
    S = sum(sig)
    mx = sum(s / S * Fraction(gx) for s, (gx, _) in zip(sig, grads))
    my = sum(s / S * Fraction(gy) for s, (_, gy) in zip(sig, grads))
    return float(A * (mx * mx + my * my)), [float(x) for x in b], [float(s) for s in sig]


def _gamma(h, t):
    """gamma_{l,m} = (1/h)^(l-1) / sum over l = 1..t (Section 3.2, Step 2)."""
    gb = [(1.0 / h) ** (l - 1) for l in range(1, t + 1)]
    return [x / sum(gb) for x in gb]


@pytest.mark.parametrize("N,top", [(1, None), (2, "cubic"), (2, "quartic"), (2, "cubic_tel"), (2, "quadratic")])
def test_sigma_beta1_tau_omega_by_value(N, top):
    M, d, U, e0, g = _piecewise_linear_case(N)
    out, info = csweno.reconstruct(d, U, [e0], return_info=True, top=top)
    P = M.V[e0]
    area = _area(P)
    sides = [math.dist(P[i], P[(i + 1) % 3]) for i in range(3)]
    h = sum(sides) / 3.0

    beta1, b1l, sig = _closed_form_beta1(area, GRADS)
    # the three beta_{1,l} differ, and sigma is far from 1/3 (the outer
    # square of eq. sigmaEqn matters)
    assert len({round(x, 12) for x in b1l}) == 3
    assert max(sig) > 10.0
    assert math.isclose(info["betas"][0][0, 0], beta1, rel_tol=1e-12)
    # dropping the outer square would give a different beta_1
    Af = Fraction(area)
    bb = [Af * (Fraction(gx) ** 2 + Fraction(gy) ** 2) for gx, gy in GRADS]
    inner = ((bb[0] - bb[1]) ** 2 + (bb[1] - bb[2]) ** 2 + (bb[2] - bb[0]) ** 2) / 3
    sig_wrong = [Fraction(1, 3) * (1 + inner / (bl + Fraction(1e-10))) for bl in bb]
    Sw = sum(sig_wrong)
    mxw = sum(s / Sw * Fraction(gx) for s, (gx, _) in zip(sig_wrong, GRADS))
    myw = sum(s / Sw * Fraction(gy) for s, (_, gy) in zip(sig_wrong, GRADS))
    assert abs(float(Af * (mxw * mxw + myw * myw)) - beta1) > 1e-3 * beta1

    betas = [beta1] + [float(info["betas"][l][0, 0]) for l in range(1, len(info["betas"]))]
    assert len({round(x, 10) for x in betas}) == len(betas)  # beta_1 != beta_2 != beta_3 (!= beta_4)
    tname = csweno.resolve_top(N, top)
    if tname == "quadratic":
        tau = (abs(betas[2] - betas[0]) ** 2 + abs(betas[2] - betas[1]) ** 2) / 4.0  # eq. tauNonlinearWeightsP1
        gam = _gamma(h, 3)
        tau_wrong = tau * 4.0 / 16.0
    else:
        tau = sum(abs(betas[3] - betas[l]) ** 2 for l in range(3)) / 16.0  # eq. tauNonlinearWeightsP2
        gam = _gamma(h, 4)  # gamma_{l,5}: four weights (t = m - 1)
        tau_wrong = tau * 16.0 / 4.0
    assert math.isclose(info["tau"][0, 0], tau, rel_tol=1e-12)
    assert not math.isclose(info["tau"][0, 0], tau_wrong, rel_tol=1e-3)
    assert np.allclose(info["gamma"][0], gam, rtol=1e-13)
    wbar = [gam[l] * (1.0 + tau / (1e-10 + betas[l])) for l in range(len(betas))]
    om = [x / sum(wbar) for x in wbar]
    for l in range(len(betas)):
        assert math.isclose(info["wbar"][l][0, 0], wbar[l], rel_tol=1e-12)
        assert math.isclose(info["omega"][l][0, 0], om[l], rel_tol=1e-12)
    # the weights moved away from the linear weights (the data are not smooth)
    assert max(abs(om[l] - gam[l]) for l in range(len(betas))) > 1e-3


def _mesh(n=6, seed=11):
    v, t = inputs.jittered_mesh(n, seed=seed)
    return Mesh(v, t, BC_TRANSMISSIVE, (1.0, 1.0))


def _interior(M):
    return np.nonzero(~np.any((M.info & (INFO_BOUNDARY | 0x3C)) != 0, axis=1))[0]


def _poly(deg):
    def f(x, y):
        v = 0.2 + 0.5 * x - 0.3 * y
        if deg >= 2:
            v = v + 0.4 * x * x - 0.2 * x * y + 0.3 * y * y
        if deg >= 3:
            v = v + 0.25 * x ** 3 - 0.1 * x * y * y + 0.15 * y ** 3
        if deg >= 4:
            v = v + 0.2 * x ** 4 - 0.3 * x * x * y * y
        return v
    return f


@pytest.mark.parametrize("N", [2, 3])
def test_cubic_reading_follows_eq_equivalentOrder3(N):
    """The literal reading of the N = 2 top member: p_4 is defined by eq.
    equivalentOrder3 from the cubic q_4 and the three weights gamma_{.,4}
    (t = 3), i.e. gamma_{1,4} p_1 + gamma_{2,4} p_2 + gamma_{3,4} p_4 = q_4
    with gamma_{l,4} computed here in closed form from the mean side h; q_4
    is the cubic least-squares fit on the 16-cell T4, so it reproduces cubic
    data exactly, and p_4 then equals p_3 on quadratic data (q_3 = q_4)."""
    M = _mesh(6)
    d = DG(M, N, 0)
    E = _interior(M)
    U = d.project(_poly(3 if N == 3 else 2))
    out, info = csweno.reconstruct(d, U, E, return_info=True, top="cubic", linear_only=True)
    assert info["top"] == "cubic"
    h = M.mean_side[E]
    gb = np.stack([np.ones_like(h), 1.0 / h, 1.0 / h ** 2], -1)
    g4 = gb / gb.sum(-1, keepdims=True)
    ps, qs = info["ps"], info["qs"]
    lhs = g4[:, 0, None, None] * ps[0] + g4[:, 1, None, None] * ps[1] + g4[:, 2, None, None] * ps[3]
    assert np.abs(lhs - qs[3]).max() < 1e-11 * max(1.0, np.abs(qs[3]).max())
    # q_4 has degree 3: its quartic coefficients are zero
    assert np.all(qs[3][:, 9:, :] == 0.0)
    if N == 2:
        # quadratic data: q_3 = q_4 = data, so p_4 = p_3
        assert np.abs(ps[3] - ps[2]).max() < 1e-9 * np.abs(ps[2]).max()


@pytest.mark.parametrize("top", ["cubic", "cubic_tel"])
def test_cubic_least_squares_level_reproduces_cubics(top):
    """q_4 (cubic, 15 rows / 9 unknowns on T4) reproduces cubic data: with
    N = 3 the data are exactly cubic on every element."""
    M = _mesh(6)
    d = DG(M, 3, 0)
    E = _interior(M)
    U = d.project(_poly(3))
    out, info = csweno.reconstruct(d, U, E, return_info=True, top=top)
    # mean-free coefficients of the data in the scaled monomials about the
    # centroid: x = x0 + h0 xi, so the cubic's Taylor coefficients times h0^k
    x0, y0, h0 = info["x0"], info["y0"], info["h0"]
    f = _poly(3)
    # evaluate q_4 at a few points of Delta0 against the data
    rs = [(-0.5, -0.5), (0.2, -0.7), (-0.8, 0.3)]
    for r, s in rs:
        x, y = d.mesh.physical_points(np.array([r]), np.array([s]), E)
        xi = (x[:, 0] - x0) / h0
        eta = (y[:, 0] - y0) / h0
        phi = np.stack([xi ** a * eta ** b for a, b in csweno.monomials(4)], -1) - info["mavg0"]
        q4 = info["fbar0"][:, 0] + np.einsum("tn,tn->t", phi, info["qs"][3][:, :, 0])
        assert np.abs(q4 - f(x[:, 0], y[:, 0])).max() < 1e-11


def test_telescoping_cubic_reproduces_cubics_with_linear_weights():
    """'cubic_tel': with omega = gamma_{.,5} the members telescope to q_4,
    so cubic data (N = 3) are reproduced by the linear-weight reconstruction;
    the literal 'cubic' reading does not telescope (its linear-weight
    combination mixes p_3 and p_4 with gamma_{.,5}) and departs from
    quadratic data by a small amount of order h^3."""
    M = _mesh(6)
    d3 = DG(M, 3, 0)
    E = _interior(M)
    U3 = d3.project(_poly(3))
    out = csweno.reconstruct(d3, U3, E, linear_only=True, top="cubic_tel")
    assert np.abs(out - U3[E]).max() < 1e-11
    d2 = DG(M, 2, 0)
    U2 = d2.project(_poly(2))
    lit = csweno.reconstruct(d2, U2, E, linear_only=True, top="cubic")
    dev = np.abs(lit - U2[E]).max()
    assert 1e-8 < dev < 1e-2


@pytest.mark.parametrize("top", ["cubic", "cubic_tel", "quartic", "quadratic"])
@pytest.mark.parametrize("eq", [0, 1])
def test_every_top_reproduces_linear_data(top, eq):
    """Linear data: every level reproduces them, all smoothness indicators
    coincide, tau = 0 and omega = gamma; each reading of the top member then
    returns the data (for 'cubic' because p_4 = p_3 and the gamma_{.,5}
    combination of p_1, p_2, p_3, p_3 sums to the data)."""
    M = _mesh(6)
    d = DG(M, 2, eq)
    if eq == 0:
        U = d.project(lambda x, y: 0.4 + 0.7 * x - 0.5 * y)
    else:
        U = d.project(lambda x, y: np.stack([1.0 + 0.2 * x - 0.1 * y, 0.3 + 0.1 * x, -0.2 + 0.05 * y,
                                             2.5 + 0.1 * x + 0.2 * y], -1))
    E = _interior(M)
    out, info = csweno.reconstruct(d, U, E, return_info=True, top=top)
    assert np.abs(out - U[E]).max() < 1e-11
    om = np.stack(info["omega"], 1)
    assert np.allclose(om, info["gamma"][:, :, None], atol=1e-9)


@pytest.mark.parametrize("top,ns", [("cubic", (32, 64)), ("cubic_tel", (32, 64))])
def test_single_application_of_cubic_tops_keeps_design_order(top, ns):
    """Smooth data, every cell troubled, N = 2: one application of the
    limiter with either cubic reading stays within O(h^3) of the exact
    solution (the design order of P2)."""
    ic = inputs.BurgersSine()
    errs = []
    for n in ns:
        v, t = inputs.jittered_mesh(n, -2, 2, -2, 2, seed=7)
        M = Mesh(v, t, BC_PERIODIC, (4.0, 4.0))
        d = DG(M, 2, 0)
        U = d.project(ic)
        L = csweno.limit(d, U, np.ones(M.K, bool), top=top)
        errs.append(d.errors(L, ic)[0])
    order = math.log(errs[0] / errs[1]) / math.log(2.0)
    assert order > 2.7, (errs, order)
