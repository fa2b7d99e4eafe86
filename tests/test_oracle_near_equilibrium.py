"""CPU pins of the oracle's near-equilibrium pieces (no GPU).

index_maxwellian is pinned by closed forms: a well-resolved Maxwellian sampled
on the index grid is its own fit (the discrete moments of a Gaussian equal the
continuous ones up to exp(-2 pi^2 var) by Poisson summation, and the tails at
the box edge are below 1e-14; FP64 summation leaves ~1e-12), the fit reproduces the mass, mean and
temperature of its input, and the degenerate cells map to zero.  The
near-equilibrium collision of a Maxwellian is then zero, and for any f it
differs from Q(f, f) only by the collision of the fitted Maxwellian.
"""
import numpy as np
import pytest

import oracle
from paper_1201_3986_amd import workloads


def _grid_maxwellian(d, n, mass, mu, var):
    idx = np.stack(np.meshgrid(*([np.arange(n, dtype=np.float64)] * d), indexing="ij"), -1)
    r2 = np.sum((idx - np.asarray(mu)) ** 2, -1)
    return mass * (2 * np.pi * var) ** (-d / 2) * np.exp(-r2 / (2 * var))


def _moments(d, n, f):
    idx = np.stack(np.meshgrid(*([np.arange(n, dtype=np.float64)] * d), indexing="ij"), -1).reshape(-1, d)
    v = np.asarray(f, np.float64).reshape(-1)
    s0 = v.sum()
    mu = idx.T @ v / s0
    var = (np.sum(idx * idx, 1) @ v / s0 - mu @ mu) / d
    return s0, mu, var


@pytest.mark.parametrize("d,n,mu,var,mass", [
    (2, 32, (15.8, 16.3), 3.0, 1.7),
    (2, 64, (30.0, 33.2), 9.0, 0.4),
    (3, 24, (11.6, 12.1, 12.4), 2.0, 2.0),
])
def test_resolved_maxwellian_is_its_own_fit(d, n, mu, var, mass):
    M = _grid_maxwellian(d, n, mass, mu, var)
    fit = oracle.index_maxwellian(d, n, M)
    assert np.max(np.abs(fit - M)) <= 1e-11 * np.max(M)


def test_fit_reproduces_moments_of_noisy_cells():
    rng = np.random.default_rng(3)
    for d, n in ((2, 32), (3, 24)):
        f = workloads.noisy_local_maxwellian(rng, d, n, 8.0, 0.05)
        M = oracle.index_maxwellian(d, n, f)
        a, b = _moments(d, n, f), _moments(d, n, M)
        assert abs(a[0] - b[0]) <= 1e-10 * a[0]
        assert np.max(np.abs(a[1] - b[1])) <= 1e-9 * n
        assert abs(a[2] - b[2]) <= 1e-9 * a[2]
        # and it is close to f: the noise is the only difference
        assert np.max(np.abs(f - M)) <= 0.06 * np.max(f)


def test_degenerate_cells_have_no_maxwellian():
    n = 16
    f = np.zeros((4, n, n))
    f[1] = -np.ones((n, n))            # negative mass
    f[2, 3, 9] = 5.0                   # zero temperature
    f[3, 3, 9] = f[3, 3, 10] = 1.0     # index temperature 1/8 <= 1/4
    M = oracle.index_maxwellian(2, n, f)
    assert np.all(M == 0.0)
    # batched call = per-cell calls
    f2 = np.stack([f[0], _grid_maxwellian(2, n, 1.0, (7.5, 8.0), 2.0)])
    Mb = oracle.index_maxwellian(2, n, f2)
    assert np.array_equal(Mb[1], oracle.index_maxwellian(2, n, f2[1]))


def test_near_equilibrium_collision_of_a_maxwellian_vanishes():
    d, n = 2, 32
    M = _grid_maxwellian(d, n, 1.0, (16.2, 15.6), 5.0)
    dirs = oracle.first_lines(d, 8)
    w = oracle.default_weights(d, 0.5, dirs)
    nt = oracle.default_ntilde(n)
    q = oracle.collide_near_equilibrium(d, n, nt, dirs, w, M)
    loss_scale = np.max(M) ** 2 * np.sum(w) * (2 * nt + 1) ** 2
    assert np.max(np.abs(q)) <= 1e-12 * loss_scale


def test_near_equilibrium_differs_from_full_by_the_fit_collision():
    d, n = 2, 16
    rng = np.random.default_rng(12)
    f = workloads.noisy_local_maxwellian(rng, d, n, 8.0, 0.05)
    dirs = oracle.first_lines(d, 8)
    w = oracle.default_weights(d, 1.0, dirs)
    nt = oracle.default_ntilde(n)
    near = oracle.collide_near_equilibrium(d, n, nt, dirs, w, f)
    full = oracle.collide(d, n, nt, dirs, w, f)
    fit = oracle.collide(d, n, nt, dirs, w, oracle.index_maxwellian(d, n, f))
    assert np.max(np.abs(near - (full - fit))) <= 1e-15 * np.max(np.abs(full)) * 10
    # the fitted Maxwellian's own collision is small against Q(f, f) (periodic-wrap residue)
    assert np.max(np.abs(fit)) <= 1e-3 * np.max(np.abs(full))
