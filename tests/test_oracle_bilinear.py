"""Pins of the oracle's bilinear operator Q(g, f) (gain g(i+k) f(i+l), loss
g(i) f(i+k+l); the consistency statement of Sec. 2.3 is written for D(g, f)).

Each test checks oracle.collide_bilinear against something fixed outside its
code: a brute-force sum over all orthogonal pairs of the box with the paper's
weight a(k) = h^(2d-1)|k|/gcd(k) (full set, Sec. 3.2), a NumPy FFT form of the
per-direction convolutions, the pseudo-spectral form of Sec. 3.1 written for
two functions (sum over K + L = I of (beta(K, L) - beta(L, L)) g~_K f~_L),
the diagonal Q(f, f), bilinearity, mass conservation and the near-equilibrium
identity Q(f, f) - Q(M, M) = Q(f - M, f) + Q(M, f - M).  g and f are drawn
independently, so an exchange of the two arguments anywhere fails.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from test_oracle_operator import loss_scale, pairs_of, rolled


def brute_full_bilinear(g, f, ntilde, h):
    d = f.ndim
    box = list(itertools.product(range(-ntilde, ntilde + 1), repeat=d))
    Q = np.zeros_like(f)
    for k in box:
        if not any(k):
            continue
        gc = 0
        for x in k:
            gc = math.gcd(gc, abs(x))
        a = h ** (2 * d - 1) * math.sqrt(sum(x * x for x in k)) / gc
        for l in box:
            if sum(x * y for x, y in zip(k, l)) != 0:
                continue
            kl = tuple(x + y for x, y in zip(k, l))
            Q += a * (rolled(g, k) * rolled(f, l) - g * rolled(f, kl))
    return Q


def fft_form_bilinear(g, f, ntilde, dirs, w):
    d, n = f.ndim, f.shape[0]
    G, F = np.fft.fftn(g), np.fft.fftn(f)
    Q = np.zeros_like(f)
    box = list(itertools.product(range(-ntilde, ntilde + 1), repeat=d))
    for e, wp in zip(dirs, w):
        M = ntilde // int(np.max(np.abs(e)))
        IK = np.zeros(f.shape)
        for m in range(-M, M + 1):
            if m:
                IK[tuple((m * e) % n)] += 1.0
        IL = np.zeros(f.shape)
        for l in box:
            if int(np.dot(l, e)) == 0:
                IL[tuple(np.array(l) % n)] += 1.0
        A, B = np.conj(np.fft.fftn(IK)), np.conj(np.fft.fftn(IL))
        line_g = np.fft.ifftn(G * A).real
        plane_f = np.fft.ifftn(F * B).real
        Q += wp * (line_g * plane_f - g * np.fft.ifftn(F * A * B).real)
    return Q


def _pair(seed, shape):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.1, 1.0, size=shape), rng.uniform(0.1, 1.0, size=shape)


@pytest.mark.parametrize("d,ntilde", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2)])
def test_full_set_equals_brute_force(d, ntilde):
    n, h = 8, 0.7
    g, f = _pair(40 + 10 * d + ntilde, (n,) * d)
    dirs = oracle.lines(d, ntilde)
    w = oracle.default_weights(d, h, dirs)
    q = oracle.collide_bilinear(d, n, ntilde, dirs, w, g, f).reshape(f.shape)
    ref = brute_full_bilinear(g, f, ntilde, h)
    swapped = brute_full_bilinear(f, g, ntilde, h)
    assert np.max(np.abs(q - ref)) <= 1e-13 * np.max(np.abs(ref))
    # the argument order matters: Q(f, g) is a different field
    assert np.max(np.abs(swapped - ref)) >= 1e-3 * np.max(np.abs(ref))


@pytest.mark.parametrize("d,n,ntilde,P", [(2, 16, 3, 8), (2, 12, 4, 13), (3, 8, 2, 8), (3, 9, 2, 5)])
def test_restricted_set_equals_fft_form(d, n, ntilde, P):
    g, f = _pair(60 + n + P, (n,) * d)
    dirs = oracle.first_lines(d, P)
    w = np.random.default_rng(61).uniform(0.2, 2.0, size=P)
    q = oracle.collide_bilinear(d, n, ntilde, dirs, w, g, f).reshape(f.shape)
    ref = fft_form_bilinear(g, f, ntilde, dirs, w)
    assert np.max(np.abs(q - ref)) <= 1e-13 * loss_scale(f, ntilde, dirs, w)


def test_pseudo_spectral_form():
    # Sec. 3.1: the Fourier form of the pair sum, with g~ at the gain's first
    # slot: Q~(g, f)_I = sum_{K+L=I} (beta(K, L) - beta(L, L)) g~_K f~_L
    d, n, nt = 2, 7, 2
    g, f = _pair(71, (n, n))
    dirs = oracle.first_lines(d, 6)
    w = np.random.default_rng(72).uniform(0.5, 1.5, size=len(dirs))
    Ks = np.array(list(itertools.product(range(n), repeat=d)))
    beta = np.zeros((len(Ks), len(Ks)), dtype=complex)
    for k, l, wp in pairs_of(d, nt, dirs, w):
        beta += wp * np.outer(np.exp(2j * np.pi * (Ks @ k) / n), np.exp(2j * np.pi * (Ks @ l) / n))
    gt = (np.fft.fftn(g) / n ** d).reshape(-1)
    ft = (np.fft.fftn(f) / n ** d).reshape(-1)
    index = {tuple(K): i for i, K in enumerate(Ks)}
    qt = np.zeros(len(Ks), dtype=complex)
    for iI, I in enumerate(Ks):
        for iK, K in enumerate(Ks):
            iL = index[tuple((I - K) % n)]
            qt[iI] += (beta[iK, iL] - beta[iL, iL]) * gt[iK] * ft[iL]
    q_ps = (np.fft.ifftn(qt.reshape(n, n)) * n ** d).real
    q = oracle.collide_bilinear(d, n, nt, dirs, w, g, f).reshape(f.shape)
    assert np.max(np.abs(q - q_ps)) <= 1e-12 * loss_scale(f, nt, dirs, w)


@pytest.mark.parametrize("d,n,ntilde,P", [(2, 16, 3, 16), (3, 8, 2, 13)])
def test_diagonal_bilinearity_mass_and_weights(d, n, ntilde, P):
    rng = np.random.default_rng(80 + d)
    g, f = _pair(81 + d, (n,) * d)
    u = rng.uniform(-1.0, 1.0, size=(n,) * d)
    dirs = oracle.first_lines(d, P)
    w = rng.uniform(0.2, 2.0, size=P)
    B = lambda a, b, ww=w: oracle.collide_bilinear(d, n, ntilde, dirs, ww, a, b).reshape(f.shape)
    scale = loss_scale(f, ntilde, dirs, w)
    # diagonal: Q(f, f) of the quadratic operator
    assert np.max(np.abs(B(f, f) - oracle.collide(d, n, ntilde, dirs, w, f).reshape(f.shape))) <= 1e-14 * scale
    # linear in each argument and in the weights
    assert np.max(np.abs(B(2.5 * g - u, f) - (2.5 * B(g, f) - B(u, f)))) <= 1e-13 * scale
    assert np.max(np.abs(B(g, 0.5 * f + u) - (0.5 * B(g, f) + B(g, u)))) <= 1e-13 * scale
    w2 = rng.uniform(0.2, 2.0, size=P)
    assert np.max(np.abs(B(g, f, w + 3 * w2) - (B(g, f) + 3 * B(g, f, w2)))) <= 1e-13 * scale
    # mass: sum_i Q(g, f)_i = 0 for any g, f (K_p is symmetric under m -> -m)
    assert abs(B(g, f).sum()) <= 1e-13 * scale * n ** d


def test_near_equilibrium_identity():
    # Q(f, f) - Q(M, M) = Q(f - M, f) + Q(M, f - M) for the cell's Maxwellian
    d, n, nt = 2, 16, 3
    rng = np.random.default_rng(90)
    i = np.arange(n) - n / 2
    M0 = np.exp(-(i[:, None] ** 2 + i[None, :] ** 2) / 8.0)
    f = M0 * (1 + 0.1 * rng.uniform(-1, 1, size=(n, n)))
    dirs = oracle.first_lines(d, 16)
    w = oracle.default_weights(d, 1.0, dirs)
    M = oracle.index_maxwellian(d, n, f)
    g = f - M
    lhs = oracle.collide_near_equilibrium(d, n, nt, dirs, w, f).reshape(f.shape)
    rhs = (oracle.collide_bilinear(d, n, nt, dirs, w, g, f)
           + oracle.collide_bilinear(d, n, nt, dirs, w, M, g)).reshape(f.shape)
    assert np.max(np.abs(lhs - rhs)) <= 1e-13 * loss_scale(f, nt, dirs, w)
