"""Pins of the type-I WENO reconstruction on the CSWENO subcell stencils
(oracle/weno_type1.py)."""
import math

import numpy as np
import pytest

from oracle import weno_type1 as w1
from oracle.dg import DG
from oracle.mesh import BC_PERIODIC, BC_TRANSMISSIVE, INFO_BOUNDARY, Mesh
from paper_2106_06280_amd import inputs


def _mesh(n=6, bc=BC_TRANSMISSIVE, seed=11):
    v, t = inputs.jittered_mesh(n, seed=seed)
    return Mesh(v, t, bc, (1.0, 1.0))


def _interior(M):
    return np.nonzero(~np.any((M.info & (INFO_BOUNDARY | 0x3C)) != 0, axis=1))[0]


@pytest.mark.parametrize("eq", [0, 1])
@pytest.mark.parametrize("N", [1, 2])
def test_every_small_stencil_reproduces_degree_N_data(N, eq):
    """Each small stencil is a least-squares fit of degree N: data of degree
    N are reproduced by every one of them, hence by the reconstruction for
    any weights (characteristic fields are linear maps of the data)."""
    M = _mesh(6)
    d = DG(M, N, eq)
    E = _interior(M)
    if eq == 0:
        f = (lambda x, y: 0.4 + 0.7 * x - 0.5 * y) if N == 1 else \
            (lambda x, y: 0.4 + 0.7 * x - 0.5 * y + 2.0 * x * x - 0.8 * x * y + 0.3 * y * y)
    else:
        f = lambda x, y: np.stack([1.0 + 0.2 * x - 0.1 * y + (0.3 * x * y if N == 2 else 0.0),
                                   0.3 + 0.1 * x + (0.1 * x * x if N == 2 else 0.0), -0.2 + 0.05 * y,
                                   2.5 + 0.1 * x + 0.2 * y + (0.2 * y * y if N == 2 else 0.0)], -1)
    U = d.project(f)
    out, info = w1.reconstruct_type1(d, U, E, return_info=True)
    assert np.abs(out - U[E]).max() < 1e-11
    # every stencil's polynomial is the same (the data), so the betas coincide
    b = np.stack(info["betas"], 0)
    assert np.allclose(b, b[0:1], rtol=1e-8, atol=1e-14)


@pytest.mark.parametrize("N", [1, 2])
def test_weights_in_closed_form(N):
    """omega_k = lambda_k / (eps + beta_k)^r / sum, with lambda = (1e5, 1, 1,
    1), eps = 1e-14, r = 4, from the betas of the oracle (closed form of
    eq. smoothnessIndicator pinned in test_oracle_csweno.py)."""
    M = _mesh(6)
    d = DG(M, N, 0)
    E = _interior(M)
    U = d.project(lambda x, y: 0.3 + 0.5 * np.sin(2 * math.pi * (x + y)) + np.where(x + 0.3 * y > 0.55, 0.8, 0.0))
    out, info = w1.reconstruct_type1(d, U, E, return_info=True)
    lam = [1e5, 1.0, 1.0, 1.0]
    for t in range(len(E)):
        bt = [float(info["betas"][k][t, 0]) for k in range(4)]
        wt = [lam[k] / (1e-14 + bt[k]) ** 4 for k in range(4)]
        for k in range(4):
            assert math.isclose(info["omega"][k][t, 0], wt[k] / sum(wt), rel_tol=1e-12)
    om = np.stack(info["omega"], 0)
    assert np.allclose(om.sum(0), 1.0, atol=1e-15)


def test_jump_takes_the_smooth_sector():
    """Data with a jump along a line: in cells whose central stencil crosses
    the jump, the weight goes to the sectors that do not (beta orders of
    magnitude smaller), and the reconstructed slope is that of the smooth
    side."""
    M = _mesh(8)
    d = DG(M, 1, 0)
    E = _interior(M)
    U = d.project(lambda x, y: 0.2 * x + np.where(x > 0.5, 1.0, 0.0))
    out, info = w1.reconstruct_type1(d, U, E, return_info=True)
    om = np.stack([o[:, 0] for o in info["omega"]], 0)  # [4, T]
    bc = info["betas"][0][:, 0]
    bs = np.stack([info["betas"][k][:, 0] for k in (1, 2, 3)], 0)
    crossing = bc > 1e3 * bs.min(axis=0)
    assert crossing.sum() > 3
    # the smoothest sector carries almost all the weight there
    best = 1 + bs[:, crossing].argmin(axis=0)
    assert np.all(om[best, np.nonzero(crossing)[0]] > 0.99)


@pytest.mark.parametrize("N,ns", [(1, (16, 32)), (2, (32, 64))])
def test_single_application_keeps_design_order(N, ns):
    ic = inputs.BurgersSine()
    errs = []
    for n in ns:
        v, t = inputs.jittered_mesh(n, -2, 2, -2, 2, seed=7)
        M = Mesh(v, t, BC_PERIODIC, (4.0, 4.0))
        d = DG(M, N, 0)
        U = d.project(ic)
        errs.append(d.errors(w1.limit_type1(d, U, np.ones(M.K, bool)), ic)[0])
    assert math.log2(errs[0] / errs[1]) > N + 1 - 0.3, errs


def test_mean_copied_and_untroubled_cells_untouched():
    M = _mesh(6, BC_PERIODIC)
    for eq in (0, 1):
        d = DG(M, 2, eq)
        ic = inputs.BurgersSine(k=2 * math.pi) if eq == 0 else inputs.FourQuadrant(seed=3)
        U = d.project(ic)
        mask = np.zeros(M.K, bool)
        mask[::3] = True
        out = w1.limit_type1(d, U, mask)
        assert np.array_equal(out[:, :, 0], U[:, :, 0])
        assert np.array_equal(out[~mask], U[~mask])
        assert not np.array_equal(out[mask], U[mask])


def test_rejects_other_degrees():
    M = _mesh(3)
    with pytest.raises(ValueError):
        w1.reconstruct_type1(DG(M, 3, 0), np.zeros((M.K, 1, 10)), [0])
