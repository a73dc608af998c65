"""Compact subcell WENO (CSWENO) limiter on triangles (Section 3.2).

For each troubled cell Delta0 (all cells read the pre-limit field; the
result goes to a new array, so the order of troubled cells is irrelevant):

1. Neighbours Delta_{f+1} across local faces f = 0, 1, 2 (Fig. 1).  A
   periodic neighbour is translated next to Delta0; on a transmissive
   boundary the neighbour is the mirror image of Delta0 across the face,
   carrying u_g(x) = u_0(Rx).
2. Each neighbour is cut into three subcells by joining its centroid G to
   its vertices (Fig. 2a): Delta_i1 = (G, w_f', w_f'+1) touches Delta0,
   Delta_i2 = (G, w_f'+1, w_f'+2), Delta_i3 = (G, w_f'+2, w_f').  For
   N >= 2, Delta_i2 and Delta_i3 are cut again by the perpendicular from G
   to their outer side (Fig. 2b), giving Delta_i2' = (G, w_f'+1, F2),
   Delta_i21 = (G, F2, w_f'+2), Delta_i3' = (G, w_f'+2, F3),
   Delta_i31 = (G, F3, w_f').
3. Subcell averages are averages of the neighbour's own DG polynomial.
4. Step 1: q_1 = mean of Delta0; q_2 (linear) on T2 = {Delta0, Delta_i1};
   q_3 (quadratic) on T3 = {Delta0, Delta_i1, Delta_i2, Delta_i3}; for
   N >= 2 also the cubic q_4 or the quartic q_5 on the 16-cell T4 (pieces
   of step 2).  Each
   has the exact mean of Delta0 and matches the other averages in the
   least-squares sense (QR), in the scaled monomials ((x-x0)/h0)^a
   ((y-y0)/h0)^b about the centroid of Delta0, h0 its mean side.
5. Step 2: equivalent polynomials (eqs. equivalentOrder0-4) with linear
   weights gamma_{l,m} = h^{-(l-1)} / sum (Section 3.2, Step 2); the
   option constant_gamma takes 10^{l-1} / sum instead, the weights of the
   reference cited there, which the paper replaces by the h-dependent ones.
6. Step 3: smoothness indicators (eq. smoothnessIndicator) of q_l,
   l >= 2, over all derivative orders 1..deg q_l; beta_1 from the three
   linear functions on each neighbour's centroid subcells (eqs. sigmaEqn,
   smoothnessIndicatorT1), lambda = 1/3, eps = 1e-10.
7. Step 4: WENO-Z style tau (eqs. tauNonlinearWeightsP1 / P2) and
   nonlinear weights (eqs. nonLinearWeightsP1 / P2).
8. Step 5: the moments 1..Np-1 are the L2 projection of
   R = sum_l omega_l p_l onto the basis (exact quadrature in place of the
   SCP points, whose tables are not available); the mean is copied.
9. Euler: the whole reconstruction is done per characteristic field with
   the eigenvectors of the x- and of the y-Jacobian at the mean of Delta0;
   the two results are averaged.

Readings where the paper is ambiguous:
the fourth member of the N >= 2 hierarchy (TOPS; the text defines a p_4
from the cubic q_4 by eq. equivalentOrder3 and a p_5 from the quartic q_5
by eq. equivalentOrder4, and then sums four members with gamma_{.,5} and
tau from beta_4):
  'cubic'      p_4 of eq. equivalentOrder3 as printed: q_4 (cubic, T4)
               minus gamma_{1,4} p_1 + gamma_{2,4} p_2, over gamma_{3,4},
               with the three weights gamma_{.,4} (t = m - 1 = 3); the
               members {p_1, p_2, p_3, p_4} are combined with gamma_{.,5}
               and beta_4 = beta(q_4);
  'cubic_tel'  q_4 in place of q_5 in eq. equivalentOrder4 (four weights,
               so that sum gamma_{l,5} p_l telescopes to q_4);
  'quartic'    eq. equivalentOrder4 with q_5 (the default for N = 3);
  'quadratic'  the three members of N = 1, {p_1, p_2, p_3}, with
               gamma_{.,3} and the tau of eq. tauNonlinearWeightsP1 (the
               default for N = 2: with every cell limited it is the only
               one of these readings whose errors fall at the order of
               Tables 1-3 under refinement; the three that build the fourth
               member on T4 diverge for Euler P2);
  'sextic'     N = 3 only: the P3 hierarchy built "in the same way" one
               level finer (Section 3.2, the remark on P3): the fourth
               member from a degree-6 least-squares level q_7 (27 scaled
               monomials) on the 30-piece stencil T5, by eq.
               equivalentOrder4 with the four weights gamma_{.,5}, beta of
               q_7 over derivative orders 1..6 and the tau of eq.
               tauNonlinearWeightsP2.  T5 cuts each neighbour into ten
               triangles fanned from its centroid G over its boundary
               divided at its vertices, at the feet F2, F3 of the N = 2 cut
               and at the midpoints of the five segments these make: each
               piece of T4 is halved by the segment from G to the midpoint
               of its outer side.
T2, T3 and beta_1 use the whole centroid subcells; by default N = 3 reuses
the N = 2 stencil and hierarchy with the quartic top; beta is taken of q_l;
sigma is read literally.

Parity status: pinned by tests/test_oracle_csweno.py (subcell tiling and
areas, perpendicular cut, least-squares reproduction of polynomials,
sum of linear weights, telescoping identity, sum of nonlinear weights,
beta in closed form, mean retained, linear data reproduced, convergence
with all cells troubled).  The choice of SCP points versus exact
projection, the N = 2/3 hierarchy reading, the beta and sigma readings
and the eigenvector scaling are 'parity unpinned' beyond design-order
convergence: no printed value separates them from the alternatives.
"""
from __future__ import annotations

import numpy as np

from . import basis, quadrature
from .dg import DG, PSI0
from .mesh import INFO_BOUNDARY
from .physics import EQ_EULER, euler_left_eigenvectors, euler_right_eigenvectors, ghost_state

EPS = 1e-10
LAMBDA1 = 1.0 / 3.0

# fourth member of the N >= 2 hierarchy (see the module docstring)
TOPS = ("cubic", "quadratic", "quartic", "cubic_tel", "sextic")
DEFAULT_TOP = {1: "quadratic", 2: "quadratic", 3: "quartic"}
TOP_DEGREE = {"quadratic": 2, "cubic": 3, "cubic_tel": 3, "quartic": 4, "sextic": 6}
# the ten pieces per neighbour of the stencil T5 of the sextic top
NAMES_T5 = [f"T5_{k}" for k in range(10)]


class RankError(ValueError):
    pass


def monomials(d):
    """Exponents (a, b) with 1 <= a+b <= d, ordered by degree."""
    return [(s - b, b) for s in range(1, d + 1) for b in range(s + 1)]


def top_degree(N):
    """Degree of the monomial space the reconstruction is written in."""
    return 2 if N == 1 else 4


def resolve_top(N, top=None, quadratic_top=False):
    """The top member used for degree N: N = 1 always has the quadratic
    q_3 on top; N >= 2 takes top (one of TOPS), else the default."""
    if N == 1:
        return "quadratic"
    if quadratic_top:
        return "quadratic"
    t = DEFAULT_TOP[N] if top is None else top
    if t not in TOPS:
        raise ValueError(f"unknown top member {t!r}")
    if t == "sextic" and N != 3:
        raise ValueError("the sextic top member is defined for N = 3")
    return t


# ---------------------------------------------------------------------------
# Geometry of the stencil
# ---------------------------------------------------------------------------

def _reflect(P, Q, X):
    d = Q - P
    t = np.sum((X - P) * d, axis=-1, keepdims=True) / np.sum(d * d, axis=-1, keepdims=True)
    F = P + t * d
    return 2.0 * F - X


def neighbour_frames(dg: DG, elems):
    """For each troubled cell and face: placed neighbour vertices W [T,3,3,2],
    shared-face index fp [T,3], element id [T,3] (-1 for a mirror ghost) and
    the shift [T,3,2] to subtract from placed coordinates before evaluating."""
    M = dg.mesh
    E = np.asarray(elems)
    T = len(E)
    V0 = M.V[E]
    W = np.zeros((T, 3, 3, 2))
    fp = np.zeros((T, 3), dtype=np.int64)
    nid = np.zeros((T, 3), dtype=np.int64)
    shift = np.zeros((T, 3, 2))
    sx_all, sy_all = M.neighbour_shift()
    for f in range(3):
        isb = (M.info[E, f] & INFO_BOUNDARY) != 0
        nb = M.nbr[E, f]
        real = ~isb
        Wr = M.V[np.where(real, nb, 0)]
        sh = np.stack([sx_all[E, f], sy_all[E, f]], axis=-1)
        Wr = Wr + sh[:, None, :]
        # mirror ghost across face f: CCW (v_{f+1}, v_f, R v_{f+2})
        P = V0[:, f]
        Q = V0[:, (f + 1) % 3]
        Rg = _reflect(P, Q, V0[:, (f + 2) % 3])
        Wg = np.stack([Q, P, Rg], axis=1)
        W[:, f] = np.where(real[:, None, None], Wr, Wg)
        fp[:, f] = np.where(real, M.neighbour_face()[E, f], 0)
        nid[:, f] = np.where(real, nb, -1)
        shift[:, f] = np.where(real[:, None], sh, 0.0)
    return W, fp, nid, shift


def pieces(W, fp, N, fine=False):
    """Subcell triangles of each placed neighbour.

    Returns dict name -> [T,3,3,2] for 'S1','S2','S3' and, for N >= 2,
    'S2p','S21','S3p','S31' and with fine = True the ten pieces of T5
    (NAMES_T5, in order around the neighbour from w_f'); also the number of
    feet that fell outside their side (split at the midpoint instead)."""
    T = W.shape[0]
    idx = np.arange(T)[:, None]
    fidx = np.arange(3)[None, :]
    wa = W[idx, fidx, fp]
    wb = W[idx, fidx, (fp + 1) % 3]
    wc = W[idx, fidx, (fp + 2) % 3]
    G = W.mean(axis=2)
    out = {
        "S1": np.stack([G, wa, wb], axis=2),
        "S2": np.stack([G, wb, wc], axis=2),
        "S3": np.stack([G, wc, wa], axis=2),
    }
    bad = 0
    if N >= 2:
        def foot(p, q):
            d = q - p
            t = np.sum((G - p) * d, axis=-1) / np.sum(d * d, axis=-1)
            outside = ~((t > 0.0) & (t < 1.0))
            t = np.where(outside, 0.5, t)
            return p + t[..., None] * d, int(outside.sum())
        F2, b2 = foot(wb, wc)
        F3, b3 = foot(wc, wa)
        bad = b2 + b3
        out["S2p"] = np.stack([G, wb, F2], axis=2)
        out["S21"] = np.stack([G, F2, wc], axis=2)
        out["S3p"] = np.stack([G, wc, F3], axis=2)
        out["S31"] = np.stack([G, F3, wa], axis=2)
        if fine:
            # the boundary of the neighbour, divided at its vertices and the
            # feet, then at the midpoints of the five segments
            ring = [wa, wb, F2, wc, F3]
            pts = []
            for k in range(5):
                p, q = ring[k], ring[(k + 1) % 5]
                pts += [p, 0.5 * (p + q)]
            for k in range(10):
                out[NAMES_T5[k]] = np.stack([G, pts[k], pts[(k + 1) % 10]], axis=2)
    return out, bad


def tri_area(P):
    return 0.5 * ((P[..., 1, 0] - P[..., 0, 0]) * (P[..., 2, 1] - P[..., 0, 1])
                  - (P[..., 2, 0] - P[..., 0, 0]) * (P[..., 1, 1] - P[..., 0, 1]))


# ---------------------------------------------------------------------------
# Averages
# ---------------------------------------------------------------------------

def neighbour_average(dg: DG, u, E, nid, shift, face, P, extrapolate=None):
    """Average of the neighbour-across-face polynomial over triangles
    P [T,3,2] (placed frame), all components: [T, m].  extrapolate [T]
    (boundary faces only): the ghost carries Delta0's own polynomial
    continued across the face instead of its mirror image."""
    M = dg.mesh
    x, y, w = quadrature.physical_rule_on_triangle(P, max(1, (dg.N + 2) // 2))
    real = nid[:, face] >= 0
    # real neighbour: undo the placement shift, map to its reference element
    nb = np.where(real, nid[:, face], E)
    xr = x - shift[:, face, 0][:, None]
    yr = y - shift[:, face, 1][:, None]
    # mirror ghost: reflect back into Delta0 and evaluate Delta0's polynomial
    V0 = M.V[E]
    Pf = V0[:, face]
    Qf = V0[:, (face + 1) % 3]
    X = np.stack([x, y], axis=-1)
    Xm = _reflect(Pf[:, None, :], Qf[:, None, :], X)
    if extrapolate is not None:
        Xm = np.where(np.asarray(extrapolate)[:, None, None], X, Xm)
    xe = np.where(real[:, None], xr, Xm[..., 0])
    ye = np.where(real[:, None], yr, Xm[..., 1])
    r, s = M.reference_coords(nb, xe, ye)
    Vh = basis.vandermonde(dg.N, r, s)  # [T, q, Np]
    vals = np.einsum("tqn,tcn->tqc", Vh, u[nb])
    if extrapolate is not None and np.any(extrapolate):
        # outside the reference triangle the collapsed coordinates of the
        # basis are singular on the line s = 1: write Delta0's polynomial in
        # the monomials r^a s^b (interpolating it at the volume points) and
        # evaluate those
        ex = np.asarray(extrapolate)
        mono = [(a, b) for d in range(dg.N + 1) for b in range(d + 1) for a in [d - b]]
        Vm = np.stack([dg.vr ** a * dg.vs ** b for a, b in mono], axis=-1)  # [q, Np]
        coef = np.linalg.lstsq(Vm, dg.V, rcond=None)[0]  # psi_n = sum_k coef[k, n] r^a_k s^b_k
        Mo = np.stack([r ** a * s ** b for a, b in mono], axis=-1)  # [T, q, Np]
        vm = np.einsum("tqk,kn,tcn->tqc", Mo, coef, u[nb])
        vals = np.where(ex[:, None, None], vm, vals)
    return np.einsum("tq,tqc->tc", w, vals) / np.sum(w, axis=1)[:, None]


def monomial_average(P, x0, y0, h0, d):
    """Average of each scaled monomial of degree 1..d over triangles P
    [T,...,3,2]: [T,..., n_mono]."""
    n = max(1, (d + 2) // 2)
    x, y, w = quadrature.physical_rule_on_triangle(P, n)
    extra = x.ndim - 2
    sh = (slice(None),) + (None,) * (extra + 1)
    xi = (x - x0[sh]) / h0[sh]
    eta = (y - y0[sh]) / h0[sh]
    cols = [np.sum(w * xi ** a * eta ** b, axis=-1) / np.sum(w, axis=-1) for a, b in monomials(d)]
    return np.stack(cols, axis=-1)


# ---------------------------------------------------------------------------
# The limiter
# ---------------------------------------------------------------------------

def linear_weights(h0, t, constant=False):
    """gamma_{l,m}, l = 1..t, normalised to sum 1: [T, t].  The paper's
    gamma_bar = (1/h)^{l-1} (Section 3.2, Step 2), or with constant = True
    gamma_bar = 10^{l-1}, the choice of the reference it cites there, which
    the paper replaces by the h-dependent one."""
    base = np.full_like(h0, 10.0) if constant else 1.0 / h0
    g = np.stack([base ** (l - 1) for l in range(1, t + 1)], axis=-1)
    return g / np.sum(g, axis=-1, keepdims=True)


def _solve_ls(A, b):
    """Least squares with QR for A [T, r, c], b [T, r, F]; asserts rank."""
    Q, R = np.linalg.qr(A)
    diag = np.abs(np.diagonal(R, axis1=-2, axis2=-1))
    if np.any(diag.min(axis=-1) <= 1e-12 * diag.max(axis=-1)):
        raise RankError("rank-deficient stencil least-squares system")
    return np.linalg.solve(R, np.einsum("trc,trf->tcf", Q, b))


def _beta_matrix(V0, x0, y0, h0, area0, d, orders=None):
    """B [T, n, n] with c^T B c = sum_{1<=|alpha|<=orders} |D0|^{|alpha|-1}
    int_D0 (D^alpha q)^2 dA for q = sum_j c_j phi_j of degree d (physical
    derivatives; orders = d unless given)."""
    mono = monomials(d)
    x, y, w = quadrature.physical_rule_on_triangle(V0, max(1, (2 * d + 2) // 2))
    xi = (x - x0[:, None]) / h0[:, None]
    eta = (y - y0[:, None]) / h0[:, None]
    T = V0.shape[0]
    B = np.zeros((T, len(mono), len(mono)))
    for s in range(1, (d if orders is None else min(d, orders)) + 1):
        for a1 in range(s + 1):
            a2 = s - a1
            # D^alpha phi_j = a!/(a-a1)! b!/(b-a2)! h0^{-s} xi^{a-a1} eta^{b-a2}
            cols = []
            for a, b in mono:
                if a < a1 or b < a2:
                    cols.append(np.zeros_like(xi))
                    continue
                coef = 1.0
                for t in range(a1):
                    coef *= (a - t)
                for t in range(a2):
                    coef *= (b - t)
                cols.append(coef * xi ** (a - a1) * eta ** (b - a2) / h0[:, None] ** s)
            D = np.stack(cols, axis=-1)  # [T, q, n]
            B += (area0 ** (s - 1))[:, None, None] * np.matmul((w[..., None] * D).transpose(0, 2, 1), D)
    return B


def reconstruct(dg: DG, u, elems, linear_only=False, return_info=False, characteristic=True, quadratic_top=False,
                constant_gamma=False, beta_literal=False, ghost_extrapolate=False, top=None):
    """New coefficients for the troubled cells elems: [T, m, Np].  Mode 0
    is copied from u.  linear_only: the weights are the linear weights
    (omega = gamma); characteristic=False (Euler): the conserved variables
    are reconstructed directly instead of the characteristic fields.
    top (N >= 2): the fourth member of the hierarchy, one of TOPS
    (default DEFAULT_TOP[N]); quadratic_top = True is top = 'quadratic',
    the hierarchy of N = 1, {p_1, p_2, p_3} with the quadratic q_3 on top
    (a third-order reconstruction: the design order of P2, one below that
    of P3).
    constant_gamma: linear weights from 10^{l-1} instead of (1/h)^{l-1}.
    beta_literal: the smoothness indicators of eq. smoothnessIndicator
    read literally, of the equivalent polynomials p_l over derivative orders
    1..N, instead of q_l over orders 1..deg q_l (a study of the reading; the
    library has no such switch).
    ghost_extrapolate: across an outflow face the ghost cell (the mirror
    image of Delta0's triangle) carries Delta0's polynomial continued across
    the face instead of its mirror image (walls keep the mirror image)."""
    M = dg.mesh
    E = np.asarray(elems, dtype=np.int64)
    T = len(E)
    N = dg.N
    m = dg.m
    Np = dg.Np
    if T == 0:
        return np.zeros((0, m, Np))
    tname = resolve_top(N, top, quadratic_top)
    dtop = max(top_degree(N), TOP_DEGREE[tname])
    V0 = M.V[E]
    x0 = V0[:, :, 0].mean(axis=1)
    y0 = V0[:, :, 1].mean(axis=1)
    h0 = M.mean_side[E]
    area0 = M.area[E]

    W, fp, nid, shift = neighbour_frames(dg, E)
    pcs, nbad = pieces(W, fp, N, fine=tname == "sextic")
    names_t3 = ["S1", "S2", "S3"]
    names_t4 = NAMES_T5 if tname == "sextic" else ["S1", "S2p", "S21", "S3p", "S31"]

    # cell averages of u (all components) on the pieces: avg[name] [T, 3, m]
    avg = {}
    for name in pcs:
        avg[name] = np.stack([neighbour_average(dg, u, E, nid, shift, f, pcs[name][:, f],
                                                extrapolate=(ghost_extrapolate
                                                             & ((M.info[E, f] & INFO_BOUNDARY) != 0)
                                                             & ((M.info[E, f] & 3) == 0)))
                              for f in range(3)], axis=1)
    # ghost cells of boundary faces carry the boundary's ghost state: the
    # mirrored polynomial (outflow), the same with its normal momentum
    # reversed (reflective wall), the inflow state on every piece (inflow),
    # the moving shock's state at the face midpoint and the solution time on
    # every piece (moving shock); averaging commutes with the reflection
    for f in range(3):
        isb = (M.info[E, f] & INFO_BOUNDARY) != 0
        if not isb.any():
            continue
        kind = np.where(isb, M.info[E, f] & 3, 0)
        xm = ym = None
        if dg.shock is not None:
            mid = 0.5 * (M.V[E, f] + M.V[E, (f + 1) % 3])
            xm, ym = mid[:, 0], mid[:, 1]
        for name in pcs:
            g = ghost_state(dg.eq, avg[name][:, f], kind, M.nx[E, f], M.ny[E, f], dg.inflow, dg.shock, xm, ym,
                            dg.time)
            avg[name][:, f] = np.where(isb[:, None], g, avg[name][:, f])
    ubar0 = u[E, :, 0] * PSI0  # [T, m]

    # scaled-monomial averages
    mono_top = monomials(dtop)
    mavg0 = monomial_average(V0, x0, y0, h0, dtop)  # [T, n]
    mavg = {name: monomial_average(pcs[name], x0, y0, h0, dtop) for name in pcs}  # [T,3,n]

    def rows(names):
        A = np.concatenate([mavg[nm] for nm in names], axis=1)  # [T, 3*len, n] ordered name-major
        return A - mavg0[:, None, :]

    def rhs(names, data, data0):
        b = np.concatenate([data[nm] for nm in names], axis=1)
        return b - data0[:, None, :]

    # characteristic transforms
    if dg.eq == EQ_EULER and not characteristic:
        Ls = [np.broadcast_to(np.eye(m), (T, m, m))]
        Rs = [np.broadcast_to(np.eye(m), (T, m, m))]
    elif dg.eq == EQ_EULER:
        Ubar = ubar0
        dirs = [(1.0, 0.0), (0.0, 1.0)]
        Ls = [euler_left_eigenvectors(Ubar, nx, ny, dg.gamma) for nx, ny in dirs]
        Rs = [euler_right_eigenvectors(Ubar, nx, ny, dg.gamma) for nx, ny in dirs]
    else:
        Ls = [np.ones((T, 1, 1))]
        Rs = [np.ones((T, 1, 1))]
    ND = len(Ls)
    # field data for all directions: F = ND * m fields
    def to_fields(a):  # a [T, k, m] -> [T, k, ND*m]
        return np.concatenate([np.einsum("tij,tkj->tki", Ls[d], a) for d in range(ND)], axis=-1)
    favg = {nm: to_fields(avg[nm]) for nm in avg}
    fbar0 = to_fields(ubar0[:, None, :])[:, 0, :]  # [T, F]
    F = ND * m

    nlin = len(monomials(1))
    nquad = len(monomials(2))
    dfour = TOP_DEGREE[tname]
    # Step 1: q_2, q_3 and the top least-squares level on T4 (the cubic
    # q_4 or the quartic q_5), or on T5 (the sextic q_7)
    c2 = _solve_ls(rows(["S1"])[:, :, :nlin], rhs(["S1"], favg, fbar0))  # [T, 2, F]
    c3 = _solve_ls(rows(names_t3)[:, :, :nquad], rhs(names_t3, favg, fbar0))  # [T, 5, F]
    ntop = len(mono_top)
    pad = lambda c: np.concatenate([c, np.zeros((T, ntop - c.shape[1], F))], axis=1)
    qs = [np.zeros((T, ntop, F)), pad(c2), pad(c3)]
    four = tname != "quadratic"
    if four:
        nfour = len(monomials(dfour))
        c4 = _solve_ls(rows(names_t4)[:, :, :nfour], rhs(names_t4, favg, fbar0))  # [T, 9, 14 or 27, F]
        qs.append(pad(c4))
    L = len(qs)

    # Step 2: equivalent polynomials (mean-free parts; all means equal ubar0)
    g2 = linear_weights(h0, 2, constant_gamma)
    g3 = linear_weights(h0, 3, constant_gamma)
    ps = [qs[0], qs[1] / g2[:, 1, None, None]]  # p1 = q1 has zero mean-free part
    ps.append((qs[2] - g3[:, 1, None, None] * ps[1]) / g3[:, 2, None, None])
    if four:
        g5 = linear_weights(h0, 4, constant_gamma)
        if tname == "cubic":
            # eq. equivalentOrder3: q_4 = gamma_{1,4} p_1 + gamma_{2,4} p_2 +
            # gamma_{3,4} p_4 with the three weights gamma_{.,4}
            g4 = linear_weights(h0, 3, constant_gamma)
            ps.append((qs[3] - g4[:, 1, None, None] * ps[1]) / g4[:, 2, None, None])
        else:
            # eq. equivalentOrder4 (q_5, q_4 in its place, or q_7)
            ps.append((qs[3] - sum(g5[:, l, None, None] * ps[l] for l in range(3))) / g5[:, 3, None, None])
        gtop = g5
    else:
        gtop = g3

    # Step 3: smoothness indicators of q_l (l >= 2)
    betas = [None]
    degs = [0, 1, 2, dfour]
    for l in range(1, L):
        d = degs[l]
        nd = len(monomials(d))
        if beta_literal:
            c = ps[l][:, :nd, :]
            Bl = _beta_matrix(V0, x0, y0, h0, area0, d, orders=N)
        else:
            c = qs[l][:, :nd, :]
            Bl = _beta_matrix(V0, x0, y0, h0, area0, d)
        betas.append(np.einsum("tif,tij,tjf->tf", c, Bl, c))
    # beta_1 from linear functions on each neighbour's centroid subcells
    cen = {nm: pcs[nm].mean(axis=2) for nm in names_t3}  # [T,3,2]
    grads = []
    b1l = []
    for f in range(3):
        Mx = np.stack([cen["S2"][:, f] - cen["S1"][:, f], cen["S3"][:, f] - cen["S1"][:, f]], axis=1)  # [T,2,2]
        rhs1 = np.stack([favg["S2"][:, f] - favg["S1"][:, f], favg["S3"][:, f] - favg["S1"][:, f]], axis=1)  # [T,2,F]
        gr = np.linalg.solve(Mx, rhs1)  # [T, 2, F]
        grads.append(gr)
        b1l.append(area0[:, None] * np.sum(gr * gr, axis=1))
    b11, b12, b13 = b1l
    num = ((np.abs(b11 - b12) ** 2 + np.abs(b12 - b13) ** 2 + np.abs(b13 - b11) ** 2) / 3.0) ** 2
    sig = [LAMBDA1 * (1.0 + num / (b + EPS)) for b in b1l]
    ssum = sig[0] + sig[1] + sig[2]
    gmix = sum((sig[f] / ssum)[:, None, :] * grads[f] for f in range(3))
    betas[0] = area0[:, None] * np.sum(gmix * gmix, axis=1)

    # Step 4: tau and nonlinear weights
    if not four:
        tau = (np.abs(betas[2] - betas[0]) ** 2 + np.abs(betas[2] - betas[1]) ** 2) / 4.0
    else:
        tau = sum(np.abs(betas[3] - betas[l]) ** 2 for l in range(3)) / 16.0
    wbar = [gtop[:, l, None] * (1.0 + tau / (EPS + betas[l])) for l in range(L)]
    if linear_only:
        wbar = [gtop[:, l, None] * np.ones_like(tau) for l in range(L)]
    wsum = sum(wbar)
    omega = [wb / wsum for wb in wbar]
    Rc = sum(omega[l][:, None, :] * ps[l] for l in range(L))  # [T, ntop, F]

    # Step 5: L2 projection of R = fbar0 + sum_j Rc_j (phi_j - avg phi_j) onto psi_i
    r, s, w = quadrature.triangle_rule_for_degree(dtop + N)
    Vh = basis.vandermonde(N, r, s)  # [q, Np]
    lam1 = 0.5 * (1.0 + r)
    lam2 = 0.5 * (1.0 + s)
    xq = V0[:, 0, 0, None] + lam1 * (V0[:, 1, 0, None] - V0[:, 0, 0, None]) + lam2 * (V0[:, 2, 0, None] - V0[:, 0, 0, None])
    yq = V0[:, 0, 1, None] + lam1 * (V0[:, 1, 1, None] - V0[:, 0, 1, None]) + lam2 * (V0[:, 2, 1, None] - V0[:, 0, 1, None])
    xi = (xq - x0[:, None]) / h0[:, None]
    eta = (yq - y0[:, None]) / h0[:, None]
    phi = np.stack([xi ** a * eta ** b for a, b in mono_top], axis=-1) - mavg0[:, None, :]  # [T,q,n]
    Rq = fbar0[:, None, :] + np.einsum("tqn,tnf->tqf", phi, Rc)  # [T, q, F]
    mom = np.einsum("q,tqf,qi->tfi", w, Rq, Vh)  # [T, F, Np]
    out = np.zeros((T, m, Np))
    for d in range(ND):
        out += np.einsum("tij,tjn->tin", Rs[d], mom[:, d * m:(d + 1) * m, :]) / ND
    out[:, :, 0] = u[E, :, 0]
    if return_info:
        return out, dict(qs=qs, ps=ps, betas=betas, omega=omega, gamma=gtop, tau=tau,
                         pieces=pcs, avg=avg, fbar0=fbar0, nbad=nbad, Rc=Rc, mavg0=mavg0,
                         x0=x0, y0=y0, h0=h0, favg=favg, top=tname, wbar=wbar, area0=area0)
    return out


def limit(dg: DG, u, mask, linear_only=False, characteristic=True, quadratic_top=False, constant_gamma=False,
          beta_literal=False, ghost_extrapolate=False, top=None):
    """Apply the limiter to the cells where mask is true (simultaneous
    update: every reconstruction reads the pre-limit u)."""
    E = np.nonzero(np.asarray(mask))[0]
    out = u.copy()
    if len(E):
        out[E] = reconstruct(dg, u, E, linear_only=linear_only, characteristic=characteristic,
                             quadratic_top=quadratic_top, constant_gamma=constant_gamma, beta_literal=beta_literal,
                             ghost_extrapolate=ghost_extrapolate, top=top)
    return out


def stencil_list(mesh, e):
    """Per face: (neighbour id or -1 for a mirror ghost, its shared face,
    x shift code, y shift code) -> 12 ints."""
    out = []
    for f in range(3):
        inf = int(mesh.info[e, f])
        if inf & INFO_BOUNDARY:
            out += [-1, 0, 0, 0]
        else:
            out += [int(mesh.nbr[e, f]), inf & 3, (inf >> 2) & 3, (inf >> 4) & 3]
    return out
