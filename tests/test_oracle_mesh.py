"""Pins for the oracle's connectivity and geometry (Section 2 eq.
triangulation; Section 3.1; Section 3.2)."""
import math

import numpy as np
import pytest

from oracle.mesh import (BC_PERIODIC, BC_TRANSMISSIVE, INFO_BOUNDARY, Mesh, MeshError,
                         connectivity, connectivity_bruteforce)
from paper_2106_06280_amd import inputs


@pytest.mark.parametrize("n", [1, 2, 3])
@pytest.mark.parametrize("bc,period", [(BC_PERIODIC, (2.0, 2.0)), (BC_TRANSMISSIVE, (2.0, 2.0)),
                                       (BC_PERIODIC, (2.0, 0.0)), (BC_PERIODIC, (0.0, 2.0))])
def test_connectivity_matches_bruteforce(n, bc, period):
    v, t = inputs.jittered_mesh(n, 0.0, 2.0, -1.0, 1.0, seed=10 + n)
    a = connectivity(v, t, bc, period)
    b = connectivity_bruteforce(v, t, bc, period)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_periodic_in_one_direction():
    """Periodic in y only (Example 4's sides): the n faces on x = 0 and the n
    on x = 1 are boundary faces, the faces on y = 0 and y = 1 are paired
    with a y shift."""
    n = 4
    v, t = inputs.jittered_mesh(n, seed=3)
    tri, nbr, info = connectivity(v, t, BC_PERIODIC, (0.0, 1.0))
    nb = (info & INFO_BOUNDARY) != 0
    assert nb.sum() == 2 * n and np.all(nbr[nb] == -1)
    mid = 0.5 * (v[tri] + v[np.roll(tri, -1, axis=1)])
    assert np.all((np.abs(mid[nb][:, 0]) < 1e-12) | (np.abs(mid[nb][:, 0] - 1.0) < 1e-12))
    cy = (info >> 4) & 3
    assert (cy != 0).sum() == 2 * n and np.all((info >> 2) & 3 == 0)


def test_connectivity_symmetric_and_shifts_cancel():
    v, t = inputs.jittered_mesh(5, seed=3)
    tri, nbr, info = connectivity(v, t, BC_PERIODIC, (1.0, 1.0))
    for e in range(tri.shape[0]):
        for f in range(3):
            e2, f2 = nbr[e, f], info[e, f] & 3
            assert nbr[e2, f2] == e and (info[e2, f2] & 3) == f
            cx, cy = (info[e, f] >> 2) & 3, (info[e, f] >> 4) & 3
            cx2, cy2 = (info[e2, f2] >> 2) & 3, (info[e2, f2] >> 4) & 3
            sgn = {0: 0, 1: 1, 2: -1}
            assert sgn[cx] == -sgn[cx2] and sgn[cy] == -sgn[cy2]


def test_transmissive_boundary_count():
    n = 4
    v, t = inputs.jittered_mesh(n, seed=3)
    _, nbr, info = connectivity(v, t, BC_TRANSMISSIVE)
    nb = (info & INFO_BOUNDARY) != 0
    assert nb.sum() == 4 * n
    assert np.all(nbr[nb] == -1)


def test_ccw_fix_and_errors():
    v, t = inputs.jittered_mesh(3, seed=4)
    t2 = t.copy()
    t2[::3, 1], t2[::3, 2] = t[::3, 2], t[::3, 1]
    a = connectivity(v, t, BC_PERIODIC, (1.0, 1.0))
    b = connectivity(v, t2, BC_PERIODIC, (1.0, 1.0))
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    bad = t.copy()
    bad[0] = [bad[0, 0], bad[0, 0], bad[0, 1]]
    with pytest.raises(MeshError):
        connectivity(v, bad, BC_TRANSMISSIVE)
    with pytest.raises(MeshError):
        connectivity(v, t, BC_PERIODIC, (1.5, 1.0))


def test_geometry_closed_form():
    v = np.array([[0.0, 0.0], [3.0, 0.0], [0.0, 4.0]])
    t = np.array([[0, 1, 2]])
    M = Mesh(v, t, BC_TRANSMISSIVE)
    assert M.area[0] == 6.0 and M.J[0] == 3.0
    assert math.isclose(M.circumradius[0], 2.5, rel_tol=1e-15)
    assert math.isclose(M.inradius[0], 1.0, rel_tol=1e-15)
    assert math.isclose(M.mean_side[0], 4.0, rel_tol=1e-15)
    # outward normals of a CCW triangle
    assert np.allclose([M.nx[0, 0], M.ny[0, 0]], [0, -1])
    assert np.allclose([M.nx[0, 2], M.ny[0, 2]], [-1, 0])
    assert np.allclose([M.nx[0, 1], M.ny[0, 1]], [0.8, 0.6])
    r, s = M.reference_coords(np.array([0]), np.array([[1.0]]), np.array([[1.0]]))
    x, y = M.physical_points(r[0], s[0])
    assert np.allclose([x[0, 0], y[0, 0]], [1.0, 1.0])
