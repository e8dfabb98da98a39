"""Seeded input generators (no method arithmetic): shapes, seeding and the
instance indexing of the freezing sweep, checked on the CPU."""
import math

import numpy as np

from paper_1707_02162_amd import workloads as W


def test_freezing_sweep_indexing_and_seeding():
    omegas, lambdas = np.linspace(1, 25, 7), np.linspace(0, 1, 5)
    full = W.freezing_sweep(omegas, lambdas, N=64)
    assert full.B == 35 and full.d == 8 and full.u.shape == (35, 64, 1)
    part = W.freezing_sweep(omegas, lambdas, N=64, first=11, count=9)
    # a slice of the grid is the same instances as the whole grid (per-instance seeds)
    assert np.array_equal(part.u, full.u[11:20])
    # instance j * n_omega + i is (omega_i, lambda_j)
    for r in range(full.B):
        assert full.meta["omega"][r] == omegas[r % 7] and full.meta["lam"][r] == lambdas[r // 7]
    # lambda = 0: the noise-free drive -h0 cos(omega t) at the segment midpoints
    h0 = 5.0 * math.pi
    t = (np.arange(64) + 0.5) * (20 * math.pi / 64)
    np.testing.assert_allclose(full.u[3, :, 0], -h0 * np.cos(omegas[3] * t), rtol=0, atol=1e-4 * h0)
    # lambda = 1: pure noise, |u| <= h0, with mean close to 0
    noise = full.u[28:, :, 0]
    assert np.abs(noise).max() <= h0 * (1 + 1e-6) and abs(noise.mean()) < 0.1 * h0
    # coarse graining of the coefficient: eps = 1e-4 h0, b = 100, P = 2
    assert full.eps == 1e-4 * h0 and full.base == 100 and full.digits == 2
    assert full.dt == 20 * math.pi / 64
