"""CPU pins of the oracle's equilibrium distance (the measure that picks a
cell's direction count in the adaptive batch; no GPU).

r = sum |f - M| / sum |f| with M the index-grid Maxwellian of f.  Pinned by
closed forms: a resolved Maxwellian is at distance 0; adding a perturbation
delta with zero mass, momentum and energy moments leaves the fitted Maxwellian
unchanged, so the distance is sum |delta| / sum |M + delta| exactly; the
distance is invariant under scaling; cells without a Maxwellian are at
distance 1 and the zero cell at 0.  The level rule counts thresholds exceeded
strictly.
"""
import numpy as np
import pytest

import oracle
from paper_1201_3986_amd import workloads


def _grid(d, n):
    return np.stack(np.meshgrid(*([np.arange(n, dtype=np.float64)] * d), indexing="ij"), -1).reshape(-1, d)


def _maxwellian(d, n, mass, mu, var):
    idx = _grid(d, n)
    r2 = np.sum((idx - np.asarray(mu)) ** 2, 1)
    return (mass * (2 * np.pi * var) ** (-d / 2) * np.exp(-r2 / (2 * var))).reshape((n,) * d)


# temperatures small enough that the tails beyond the box edge are below 1e-14
@pytest.mark.parametrize("d,n,mu,var", [(2, 32, (15.3, 16.8), 3.0), (3, 24, (11.5, 12.2, 11.9), 2.0)])
def test_resolved_maxwellian_is_at_distance_zero(d, n, mu, var):
    M = _maxwellian(d, n, 1.3, mu, var)
    assert oracle.equilibrium_distance(d, n, M)[0] <= 1e-10


@pytest.mark.parametrize("d,n,mu,var", [(2, 32, (15.3, 16.8), 3.0), (3, 24, (11.6, 12.1, 11.9), 2.0)])
def test_moment_free_perturbation_gives_closed_form(d, n, mu, var):
    M = _maxwellian(d, n, 0.9, mu, var)
    idx = _grid(d, n)
    B = np.column_stack([np.ones(len(idx))] + [idx[:, k] for k in range(d)] + [np.sum(idx * idx, 1)])
    rng = np.random.default_rng(5)
    delta = rng.standard_normal(len(idx))
    delta -= B @ np.linalg.solve(B.T @ B, B.T @ delta)     # zero mass, momentum and energy moments
    assert np.max(np.abs(B.T @ delta)) <= 1e-9 * np.sum(np.abs(delta)) * n * n
    delta *= 1e-3 * M.max() / np.max(np.abs(delta))
    f = M + delta.reshape(M.shape)
    expect = np.sum(np.abs(delta)) / np.sum(np.abs(f))
    got = oracle.equilibrium_distance(d, n, f)[0]
    assert abs(got - expect) <= 1e-6 * expect


def test_scale_invariance_and_batch():
    f, _ = workloads.relaxation_mix(3, 8, 2, 16)
    r = oracle.equilibrium_distance(2, 16, f)
    # a power of two scales every sum exactly; another factor to FP64 rounding
    # (amplified where f - M cancels to ~1e-3 of f)
    assert np.array_equal(oracle.equilibrium_distance(2, 16, 4.0 * f.astype(np.float64)), r)
    assert np.allclose(oracle.equilibrium_distance(2, 16, 3.7 * f.astype(np.float64)), r, rtol=1e-10, atol=0)
    for c in range(len(f)):
        assert oracle.equilibrium_distance(2, 16, f[c])[0] == r[c]


def test_cells_without_maxwellian():
    n = 16
    f = np.zeros((3, n, n))
    f[1] = -workloads.random_positive(2, 2, n, 1)[0]      # negative mass
    f[2, 4, 4], f[2, 4, 5], f[2, 5, 4] = 2.0, 1.0, 1.0      # index temperature 3/16 <= 1/4
    r = oracle.equilibrium_distance(2, n, f)
    assert r[0] == 0.0 and r[1] == 1.0 and r[2] == 1.0


def test_levels_count_thresholds_strictly():
    thr = np.array([0.004, 0.04], np.float32)
    t0, t1 = float(thr[0]), float(thr[1])
    r = np.array([0.0, t0, np.nextafter(t0, 1.0), 0.02, t1, 0.5])
    assert list(oracle.adaptive_levels(r, thr)) == [0, 0, 1, 1, 1, 2]
    assert list(oracle.adaptive_levels(r, [])) == [0] * 6


def test_relaxation_mix_separates_by_kind():
    # the workload's kinds sit in separate bands of distance, so thresholds
    # between the bands give unambiguous levels
    f, kind = workloads.relaxation_mix(11, 24, 2, 32)
    r = oracle.equilibrium_distance(2, 32, f)
    assert r[kind == 0].max() < 0.004 < r[kind == 1].min()
    assert r[kind == 1].max() < 0.04 < r[kind == 2].min()
