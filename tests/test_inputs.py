"""Seeded input generators (CPU)."""
import math

import numpy as np

from paper_2106_06280_amd import inputs


def test_batch_instances_are_seeded_and_in_range():
    a = inputs.batch_instances()
    b = inputs.batch_instances()
    assert len(a) == 256
    assert [d["n"] for d in a] == [d["n"] for d in b]
    assert [d["mesh_seed"] for d in a] == [d["mesh_seed"] for d in b]
    K = np.array([2 * d["n"] ** 2 for d in a])
    # log-uniform draws in [2000, 60000], rounded to 2 n^2
    n_lo, n_hi = math.sqrt(2000 / 2) - 0.5, math.sqrt(60000 / 2) + 0.5
    assert all(n_lo <= d["n"] <= n_hi for d in a)
    assert [d["eq"] for d in a] == [0] * 128 + [1] * 128
    assert [d["bc"] for d in a] == [0] * 128 + [1] * 128
    assert 3.5e6 < K.sum() < 5.5e6
    # the half-plane jump crosses the unit square and the Euler states are physical
    x, y = np.meshgrid(np.linspace(0, 1, 41), np.linspace(0, 1, 41))
    for d in a[::17]:
        v = d["ic"](x, y)
        if d["eq"] == 1:
            rho = v[..., 0]
            p = 0.4 * (v[..., 3] - 0.5 * (v[..., 1] ** 2 + v[..., 2] ** 2) / rho)
            assert rho.min() > 0.5 and p.min() > 0.5
        ic = d["ic"]
        side = x * ic.nx + y * ic.ny > ic.s
        assert side.any() and (~side).any()
