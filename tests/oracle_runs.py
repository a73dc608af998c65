"""Small driver around the oracle used by the convergence tests."""
import math

import numpy as np

from oracle import csweno
from oracle.dg import DG
from oracle.mesh import BC_PERIODIC, Mesh
from paper_2106_06280_amd import inputs


def load_orders():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_orders.txt")
    out = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        t, d, a, b = line.split()
        out[(int(t), int(d))] = (float(a), float(b))
    return out


def run(dg: DG, u, t_end, limit_all=False, cfl=None):
    dt0 = dg.max_dt(u, cfl)
    nsteps = int(math.ceil(t_end / dt0))
    dt = t_end / nsteps
    lim = None
    if limit_all:
        lim = lambda v: csweno.limit(dg, v, np.ones(dg.mesh.K, dtype=bool))
        u = lim(u)
    for _ in range(nsteps):
        u = dg.ssprk3_step(u, dt, lim)
    return u


def convergence(problem, N, ns, t_end, limit_all, seed=7):
    errs = []
    for n in ns:
        if problem == "burgers":
            v, t = inputs.jittered_mesh(n, -2, 2, -2, 2, seed=seed)
            M = Mesh(v, t, BC_PERIODIC, (4.0, 4.0))
            ic = inputs.BurgersSine()
            dg = DG(M, N, 0)
            u = dg.project(ic)
            u = run(dg, u, t_end, limit_all)
            errs.append(dg.errors(u, lambda x, y: ic.exact(x, y, t_end))[0])
        elif problem == "entropy":
            v, t = inputs.jittered_mesh(n, 0, 2, 0, 2, seed=seed)
            M = Mesh(v, t, BC_PERIODIC, (2.0, 2.0))
            ic = inputs.EntropyWave()
            dg = DG(M, N, 1)
            u = dg.project(ic)
            u = run(dg, u, t_end, limit_all)
            errs.append(dg.errors(u, lambda x, y: ic.exact(x, y, t_end))[0])
        elif problem == "vortex":
            v, t = inputs.jittered_mesh(n, 0, 10, -5, 5, seed=seed)
            M = Mesh(v, t, BC_PERIODIC, (10.0, 10.0))
            ic = inputs.IsentropicVortex(period_x=10.0, period_y=10.0)
            dg = DG(M, N, 1)
            u = dg.project(ic)
            u = run(dg, u, t_end, limit_all)
            errs.append(dg.errors(u, lambda x, y: ic.exact(x, y, t_end))[0])
    orders = [math.log(errs[i] / errs[i + 1]) / math.log(ns[i + 1] / ns[i]) for i in range(len(ns) - 1)]
    return errs, orders
