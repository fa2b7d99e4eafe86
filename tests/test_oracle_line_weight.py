"""Pins of the oracle's delta line-weight profile: the term of k = m e_p
carries w_p / |m|, with default w_p = h^(2d-2), i.e. a(k) = h^(2d-2)/gcd(k),
the lattice quadrature of delta(x . y) in the Carleman form for a constant
kernel (a lattice point of the line or plane orthogonal to k stands for a
length or area h^(d-1)|k|/gcd(k), and the delta contributes 1/|x| = 1/(h|k|)).

Checked against a brute-force sum over all orthogonal pairs of the box with
that weight written directly as h^(2d-2)/gcd(k) (no direction machinery), a
NumPy FFT form with the weighted line indicator, the conservation invariants
and equilibrium (which hold for any positive weights), and central
differences of the VJP.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_1201_3986_amd import workloads
from test_oracle_operator import loss_scale, rolled


def brute_full_delta(f, ntilde, h):
    d = f.ndim
    box = list(itertools.product(range(-ntilde, ntilde + 1), repeat=d))
    Q = np.zeros_like(f)
    for k in box:
        if not any(k):
            continue
        g = 0
        for x in k:
            g = math.gcd(g, abs(x))
        a = h ** (2 * d - 2) / g
        for l in box:
            if sum(x * y for x, y in zip(k, l)) != 0:
                continue
            kl = tuple(x + y for x, y in zip(k, l))
            Q += a * (rolled(f, k) * rolled(f, l) - f * rolled(f, kl))
    return Q


def fft_form_delta(f, ntilde, dirs, w):
    d, n = f.ndim, f.shape[0]
    F = np.fft.fftn(f)
    Q = np.zeros_like(f)
    box = list(itertools.product(range(-ntilde, ntilde + 1), repeat=d))
    for e, wp in zip(dirs, w):
        M = ntilde // int(np.max(np.abs(e)))
        IK = np.zeros(f.shape)
        for m in range(-M, M + 1):
            if m:
                IK[tuple((m * e) % n)] += 1.0 / abs(m)
        IL = np.zeros(f.shape)
        for l in box:
            if int(np.dot(l, e)) == 0:
                IL[tuple(np.array(l) % n)] += 1.0
        A, B = np.conj(np.fft.fftn(IK)), np.conj(np.fft.fftn(IL))
        Q += wp * (np.fft.ifftn(F * A).real * np.fft.ifftn(F * B).real - f * np.fft.ifftn(F * A * B).real)
    return Q


@pytest.mark.parametrize("d,ntilde", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2)])
def test_full_set_equals_brute_force(d, ntilde):
    n, h = 8, 0.7
    f = np.random.default_rng(140 + 10 * d + ntilde).uniform(0.1, 1.0, size=(n,) * d)
    dirs = oracle.lines(d, ntilde)
    w = oracle.default_weights(d, h, dirs, line_weight=1)
    assert np.allclose(w, h ** (2 * d - 2), rtol=1e-15)
    q = oracle.collide(d, n, ntilde, dirs, w, f, line_weight=1).reshape(f.shape)
    ref = brute_full_delta(f, ntilde, h)
    assert np.max(np.abs(q - ref)) <= 1e-13 * np.max(np.abs(ref))
    # the uniform profile is a different operator whenever a line has |m| > 1
    if ntilde > 1:
        qu = oracle.collide(d, n, ntilde, dirs, w, f).reshape(f.shape)
        assert np.max(np.abs(qu - ref)) >= 1e-3 * np.max(np.abs(ref))


@pytest.mark.parametrize("d,n,ntilde,P", [(2, 16, 3, 8), (2, 12, 4, 13), (3, 8, 2, 8)])
def test_restricted_set_equals_fft_form(d, n, ntilde, P):
    rng = np.random.default_rng(150 + n + P)
    f = rng.uniform(0.0, 1.0, size=(n,) * d)
    dirs = oracle.first_lines(d, P)
    w = rng.uniform(0.2, 2.0, size=P)
    q = oracle.collide(d, n, ntilde, dirs, w, f, line_weight=1).reshape(f.shape)
    ref = fft_form_delta(f, ntilde, dirs, w)
    assert np.max(np.abs(q - ref)) <= 1e-13 * loss_scale(f, ntilde, dirs, w)
    # the per-direction terms and the bilinear form use the same profile
    terms = oracle.collide_terms(d, n, ntilde, dirs, f, line_weight=1)
    assert np.max(np.abs(w @ terms - q.reshape(-1))) <= 1e-13 * loss_scale(f, ntilde, dirs, w)
    qb = oracle.collide_bilinear(d, n, ntilde, dirs, w, f, f, line_weight=1).reshape(f.shape)
    assert np.max(np.abs(qb - q)) <= 1e-14 * loss_scale(f, ntilde, dirs, w)


@pytest.mark.parametrize("d,n,ntilde,P,rho", [(2, 16, 3, 16, 4.5), (3, 12, 2, 13, 2.9)])
def test_conservation_and_equilibrium(d, n, ntilde, P, rho):
    rng = np.random.default_rng(160 + d)
    idx = np.stack(np.meshgrid(*([np.arange(n)] * d), indexing="ij"), axis=-1) - n // 2
    r2 = np.sum(idx.astype(float) ** 2, axis=-1)
    f = np.where(r2 < rho * rho, rng.uniform(0.2, 1.0, size=r2.shape), 0.0)
    dirs = oracle.first_lines(d, P)
    w = rng.uniform(0.5, 1.5, size=P)
    q = oracle.collide(d, n, ntilde, dirs, w, f, line_weight=1).reshape(f.shape)
    for phi in [np.ones(f.shape)] + [idx[..., a].astype(float) for a in range(d)] + [r2]:
        assert abs(np.sum(phi * q)) <= 1e-13 * np.sum(np.abs(phi * q))
    M = workloads.maxwellian(d, n, 8.0, 1.3, [0.4] + [0.0] * (d - 1), 0.45 * (16.0 / n) ** 2)
    qm = oracle.collide(d, n, ntilde, dirs, w, M, line_weight=1)
    assert np.max(np.abs(qm)) <= 1e-13 * loss_scale(M, ntilde, dirs, w)


def test_vjp_central_differences():
    d, n, ntilde, P = 2, 10, 3, 8
    rng = np.random.default_rng(170)
    f = rng.uniform(0.1, 1.0, size=(2, n, n))
    c = rng.standard_normal(f.shape)
    dirs = oracle.first_lines(d, P)
    w = rng.uniform(0.2, 1.5, P)
    gf, gw = oracle.vjp(d, n, ntilde, dirs, w, f, c, line_weight=1)
    J = lambda ff, ww: float(np.sum(c.reshape(-1) * oracle.collide(d, n, ntilde, dirs, ww, ff, line_weight=1).reshape(-1)))
    hstep = 1e-3
    for _ in range(3):
        delta = rng.standard_normal(f.shape)
        fd = (J(f + hstep * delta, w) - J(f - hstep * delta, w)) / (2 * hstep)
        an = float(np.sum(gf.reshape(-1) * delta.reshape(-1)))
        assert abs(fd - an) <= 1e-9 * (abs(an) + np.abs(gf).sum())
    for p in range(P):
        dw = np.zeros(P)
        dw[p] = 1.0
        fd = (J(f, w + hstep * dw) - J(f, w - hstep * dw)) / (2 * hstep)
        assert abs(fd - gw[p]) <= 1e-10 * (abs(gw[p]) + np.abs(gw).sum())
