"""DG spatial operator, time step and SSP-RK3 (Section 2 and the time
discretisation at the end of Section 3).

Readings (the paper prints a structured-mesh/1D form of the weak form and
'f_hat_n = f(u_hat_n)', which has no meaning for a modal basis):

* the flux is integrated by quadrature of F(u_h) (volume) and of the
  Lax-Friedrichs flux of the two traces (edges), with alpha local to each
  edge point (the larger normal wave speed of the two traces) or, with
  `DG.lf_mode = 1`, one global constant per residual: the largest
  cell-mean wave speed of the state;
* L(u)_i = (1/J) [ sum_q w_q J grad(psi_i).F(u_h)(x_q)
                   - sum_f (L_f/2) sum_g w_g psi_i(x_g) F*.n_f ];
  with the orthonormal basis the mass matrix is J I (eq. massMatrix2D), so
  its inverse is the factor 1/J;
* the neighbour traverses a shared edge in the opposite direction, so
  Gauss point g of one side meets point n_e-1-g of the other;
* boundary faces (Section 4, Examples 4-6): outflow / transmissive, the
  exterior trace equals the interior trace; reflective wall, the interior
  trace with its normal momentum reversed; inflow, a prescribed state
  (`DG.inflow`);
* time step dt = CFL * min_e(2 r_e) / a_max with r_e the inradius and a_max
  the largest cell-mean wave speed; CFL defaults to 0.3/(2N+1).

The coefficient array layout here is [K, m, Np] (element-major).

Parity status: pinned by tests/test_oracle_dg.py (exactness on global
polynomials with transmissive boundaries, freestream, conservation, RK3
stability polynomial, convergence orders of Tables 1-3 without limiter).
"""
from __future__ import annotations

import math

import numpy as np

from . import basis, quadrature
from .mesh import Mesh
from .physics import EQ_BURGERS, EQ_EULER, cell_mean_speed, flux, ghost_state, lax_friedrichs, n_vars

# Section 3.2, table:tvd (order 3): u^(i) = sum_l alpha_il u^(l) + beta_il dt L(u^(l))
RK3_ALPHA = [[1.0], [0.75, 0.25], [1.0 / 3.0, 0.0, 2.0 / 3.0]]
RK3_BETA = [[1.0], [0.0, 0.25], [0.0, 0.0, 2.0 / 3.0]]

PSI0 = 1.0 / math.sqrt(2.0)  # constant mode of the orthonormal basis


def rk_stage(i, stages, dt, residual, limiter=None):
    """Stage i (1..3) of the table:tvd RK3 from the stored stages
    [u^(0) .. u^(i-1)], followed by the limiter (Section 3.2, end)."""
    out = np.zeros_like(stages[0])
    for l, (a, b) in enumerate(zip(RK3_ALPHA[i - 1], RK3_BETA[i - 1])):
        if a != 0.0:
            out = out + a * stages[l]
        if b != 0.0:
            out = out + b * dt * residual(stages[l])
    if limiter is not None:
        out = limiter(out)
    return out


def ssprk3_step(u, dt, residual, limiter=None):
    stages = [u]
    for i in (1, 2, 3):
        stages.append(rk_stage(i, stages, dt, residual, limiter))
    return stages[-1]


class DG:
    def __init__(self, mesh: Mesh, N: int, eq: int, gamma: float = 1.4):
        self.mesh, self.N, self.eq, self.gamma = mesh, N, eq, gamma
        self.m = n_vars(eq)
        self.Np = basis.n_modes(N)
        r, s, w = quadrature.triangle_rule(quadrature.volume_points(N))
        self.vr, self.vs, self.vw = r, s, w
        self.V = basis.vandermonde(N, r, s)  # [q, Np]
        self.Dr, self.Ds = basis.grad_vandermonde(N, r, s)
        t, tw = quadrature.edge_rule(N)
        self.et, self.ew = t, tw
        self.PF = np.stack([basis.vandermonde(N, *quadrature.face_reference_points(f, t)) for f in range(3)])  # [3, g, Np]
        self.inflow = np.zeros(self.m)  # state of inflow boundary faces (conserved variables)
        # Lax-Friedrichs constant (end of Section 2): 0 local per point (the
        # default reading), 1 one global constant per residual, the largest
        # cell-mean wave speed of the state (the bound the time step uses)
        self.lf_mode = 0
        # moving planar shock of boundary kind 3 (Example 5's top boundary):
        # dict(n, d0, w, post, pre) of physics.moving_shock_state, and the
        # solution time; a step evaluates the residual of its stages at
        # t, t + dt and t + dt/2 and the limiter at t, then advances t
        self.shock = None
        self.time = 0.0

    # ------------------------------------------------------------------
    def project(self, fn, degree=None, elems=None):
        """L2 projection of fn(x, y) -> [K, q] or [K, q, m] onto the basis
        with a collapsed rule exact to degree 2N+6 (for the elements in
        elems only when given)."""
        if degree is None:
            degree = 2 * self.N + 6
        r, s, w = quadrature.triangle_rule_for_degree(degree)
        Vh = basis.vandermonde(self.N, r, s)
        x, y = self.mesh.physical_points(r, s, elems)
        vals = np.asarray(fn(x, y), dtype=np.float64)
        if vals.ndim == 2:
            vals = vals[..., None]
        # (1/J) int u psi_n dA = sum_q w_q u(x_q) psi_n(q)
        return np.einsum("q,kqc,qn->kcn", w, vals, Vh)

    def evaluate(self, u, r, s):
        """u_h at reference points (r, s) of every element: [K, q, m]."""
        Vh = basis.vandermonde(self.N, r, s)
        return np.einsum("qn,kcn->kqc", Vh, u)

    def cell_means(self, u):
        return u[:, :, 0] * PSI0

    # ------------------------------------------------------------------
    def residual(self, u, elems=None, t=None):
        """L(u) for the elements in elems (all if None): [len, m, Np]; t is
        the time of u for the moving-shock boundary (self.time if None)."""
        M = self.mesh
        t = self.time if t is None else t
        E = np.arange(M.K) if elems is None else np.asarray(elems)
        ue = u[E]
        # volume term: sum_q w_q (dpsi/dr (r_x f + r_y g) + dpsi/ds (s_x f + s_y g))
        uq = np.einsum("qn,kcn->kqc", self.V, ue)
        fq, gq = flux(self.eq, uq, self.gamma)
        rx, ry, sx, sy = (a[E][:, None, None] for a in (M.rx, M.ry, M.sx, M.sy))
        Fr = rx * fq + ry * gq
        Fs = sx * fq + sy * gq
        vol = np.einsum("q,qi,kqc->kci", self.vw, self.Dr, Fr) + np.einsum("q,qi,kqc->kci", self.vw, self.Ds, Fs)
        # surface term
        surf = np.zeros_like(vol)
        PFrev = self.PF[:, ::-1, :]
        fprime = M.neighbour_face()
        bnd = M.boundary_mask()
        a_glob = None
        if self.lf_mode == 1:
            a_glob = float(np.max(cell_mean_speed(self.eq, self.cell_means(u), self.gamma)))
        for f in range(3):
            um = np.einsum("gn,kcn->kgc", self.PF[f], ue)
            nb = M.nbr[E, f]
            isb = bnd[E, f]
            nb_safe = np.where(isb, E, nb)
            sel = PFrev[np.where(isb, 0, fprime[E, f])]  # [k, g, n]; boundary faces: unused
            up = np.einsum("kgn,kcn->kgc", sel, u[nb_safe])
            nx = np.broadcast_to(M.nx[E, f][:, None], um.shape[:2])
            ny = np.broadcast_to(M.ny[E, f][:, None], um.shape[:2])
            kind = np.broadcast_to((M.info[E, f] & 3)[:, None], um.shape[:2])
            xg = yg = None
            if self.shock is not None:
                xg, yg = M.physical_points(*quadrature.face_reference_points(f, self.et), elems=E)
            up = np.where(isb[:, None, None], ghost_state(self.eq, um, kind, nx, ny, self.inflow, self.shock, xg, yg, t),
                          up)
            Fn = lax_friedrichs(self.eq, um, up, nx, ny, self.gamma, a_glob)
            scale = M.L[E, f] / (2.0 * M.J[E])
            surf += scale[:, None, None] * np.einsum("g,gi,kgc->kci", self.ew, self.PF[f], Fn)
        return vol - surf

    # ------------------------------------------------------------------
    def max_dt(self, u, cfl=None):
        if cfl is None:
            cfl = 0.3 / (2 * self.N + 1)
        amax = np.max(cell_mean_speed(self.eq, self.cell_means(u), self.gamma))
        hmin = np.min(2.0 * self.mesh.inradius)
        return cfl * hmin / amax

    def rk_stage(self, i, stages, dt, limiter=None):
        return rk_stage(i, stages, dt, self.residual, limiter)

    def ssprk3_step(self, u, dt, limiter=None):
        """One step from self.time: the residual of stage i's input at
        t + c dt with c = 0, 1, 1/2 (the times of u^n, u^(1), u^(2)); then
        self.time advances by dt."""
        stages = [u]
        t0 = self.time
        for i, c in zip((1, 2, 3), (0.0, 1.0, 0.5)):
            stages.append(rk_stage(i, stages, dt, lambda v, c=c: self.residual(v, t=t0 + c * dt), limiter))
        self.time = t0 + dt
        return stages[-1]

    def ssprk3_step_decisions(self, u, dt, indicator, limit):
        """One step with the limiter limit(w, mask) applied to the cells
        indicator(w) marks at each stage; returns (u^{n+1}, masks), the three
        stages' troubled sets (the step's decisions, with dt)."""
        masks = []

        def lim(w):
            m = np.asarray(indicator(w), dtype=bool)
            masks.append(m)
            return limit(w, m)
        return self.ssprk3_step(u, dt, lim), masks

    def ssprk3_step_frozen(self, u, dt, masks, limit):
        """One step with dt and the three stages' troubled sets fixed: the map
        whose derivative an adjoint with frozen decisions differentiates."""
        it = iter(masks)
        return self.ssprk3_step(u, dt, lambda w: limit(w, next(it)))

    # ------------------------------------------------------------------
    def errors(self, u, exact_fn, component=0, degree=None):
        """(L1, Linf) of u_h - exact over the domain (L1 divided by |D|)."""
        if degree is None:
            degree = 2 * self.N + 6
        r, s, w = quadrature.triangle_rule_for_degree(degree)
        x, y = self.mesh.physical_points(r, s)
        uh = self.evaluate(u, r, s)[..., component]
        ex = np.asarray(exact_fn(x, y), dtype=np.float64)
        if ex.ndim == 3:
            ex = ex[..., component]
        err = np.abs(uh - ex)
        J = self.mesh.J[:, None]
        l1 = np.sum(J * w * err) / np.sum(self.mesh.area)
        return l1, float(err.max())
