"""Seeded synthetic inputs with the shapes of the paper's workloads.

This module holds no arithmetic of the collision method: it only samples
distribution functions on the velocity grid and draws random numbers.  It is
shared by the tests, the benchmark and the checks against the oracle.

Grid convention: n points per axis on [-R, R)^d, v_j = -R + j h, h = 2R / n,
arrays in C order (last axis fastest).  The Maxwellian is
M(rho, u, T)(v) = rho (2 pi T)^(-d/2) exp(-|v - u|^2 / (2T)) (Sec. 2.1).

Workloads (random draws in the order listed, numpy default_rng(seed)):

* ``c1`` (seed 101): 2D, n = 16, R = 8; f = M(1, c1, T1) + M(1, c2, T2),
  T_j ~ U[0.5, 1.5], c_j ~ U[-2, 2]^2 (draw T1, c1, T2, c2).
* ``c2`` (seed 102): 2D, n = 64, R = 8; the c1 family, then multiplied by
  (1 + 0.05 xi), xi ~ U[-1, 1] i.i.d. per point.
* ``c3`` (seed 103): 3D, n = 32, R = 8; f = sum_{j=1..3} (1/3) N(c_j, S_j),
  S_j = O_j diag(lambda_j) O_j^T, lambda_j ~ U[0.3, 2]^3, O_j Haar-distributed
  (QR of a standard normal 3x3 with the sign of diag(R) folded in),
  c_j ~ U[-1.5, 1.5]^3 (draw lambda_j, O_j, c_j per component).
* ``c4`` (seed 104): 4096 cells 2D n = 32 then 512 cells 3D n = 24, R = 8;
  per cell M(rho ~ U[0.5, 2], u ~ U[-1, 1]^d, T ~ U[0.5, 1.5]) * (1 + 0.02 xi).
* ``c5`` (seed 105): 64 cells 3D n = 32, R = 8, each drawn from the c3 family;
  cotangent ~ N(0, 1) per point.

* ``bkw`` (no randomness): the BKW solution of the 2D Maxwell gas (Sec. 4)
  sampled on the grid at time t, the accuracy study's initial data and exact
  reference.

The paper gives no public dataset; its only workload is the analytic BKW
solution of the 2D Maxwell gas (Sec. 4).  The random families stand in for it
with the same grids and box sizes.
"""
from __future__ import annotations

import numpy as np


def velocity_axes(d: int, n: int, R: float):
    h = 2.0 * R / n
    v = -R + h * np.arange(n, dtype=np.float64)
    return np.meshgrid(*([v] * d), indexing="ij")


def maxwellian(d: int, n: int, R: float, rho: float, u, T: float) -> np.ndarray:
    vs = velocity_axes(d, n, R)
    r2 = sum((vs[a] - u[a]) ** 2 for a in range(d))
    return rho * (2.0 * np.pi * T) ** (-d / 2.0) * np.exp(-r2 / (2.0 * T))


def gaussian(d: int, n: int, R: float, mean, cov) -> np.ndarray:
    vs = velocity_axes(d, n, R)
    x = np.stack([vs[a] - mean[a] for a in range(d)], axis=-1)
    inv = np.linalg.inv(cov)
    quad = np.einsum("...i,ij,...j->...", x, inv, x)
    norm = (2.0 * np.pi) ** (-d / 2.0) / np.sqrt(np.linalg.det(cov))
    return norm * np.exp(-0.5 * quad)


def haar_rotation(rng, d: int) -> np.ndarray:
    a = rng.standard_normal((d, d))
    q, r = np.linalg.qr(a)
    return q * np.sign(np.diag(r))[None, :]


def _two_maxwellians(rng, d, n, R):
    f = np.zeros((n,) * d)
    for _ in range(2):
        T = rng.uniform(0.5, 1.5)
        c = rng.uniform(-2.0, 2.0, size=d)
        f += maxwellian(d, n, R, 1.0, c, T)
    return f


def _three_gaussians(rng, d, n, R):
    f = np.zeros((n,) * d)
    for _ in range(3):
        lam = rng.uniform(0.3, 2.0, size=d)
        O = haar_rotation(rng, d)
        c = rng.uniform(-1.5, 1.5, size=d)
        f += gaussian(d, n, R, c, O @ np.diag(lam) @ O.T) / 3.0
    return f


def c1(seed: int = 101) -> dict:
    rng = np.random.default_rng(seed)
    f = _two_maxwellians(rng, 2, 16, 8.0)
    return dict(d=2, n=16, R=8.0, farey_order=4, f=f.astype(np.float32))


def c2(seed: int = 102, n: int = 64) -> dict:
    rng = np.random.default_rng(seed)
    f = _two_maxwellians(rng, 2, n, 8.0)
    f = f * (1.0 + 0.05 * rng.uniform(-1.0, 1.0, size=f.shape))
    return dict(d=2, n=n, R=8.0, f=f.astype(np.float32))


def c3(seed: int = 103, n: int = 32) -> dict:
    rng = np.random.default_rng(seed)
    f = _three_gaussians(rng, 3, n, 8.0)
    return dict(d=3, n=n, R=8.0, f=f.astype(np.float32))


def noisy_local_maxwellian(rng, d, n, R, noise=0.02):
    rho = rng.uniform(0.5, 2.0)
    u = rng.uniform(-1.0, 1.0, size=d)
    T = rng.uniform(0.5, 1.5)
    f = maxwellian(d, n, R, rho, u, T)
    return f * (1.0 + noise * rng.uniform(-1.0, 1.0, size=f.shape))


def c4(seed: int = 104, n2d_cells: int = 4096, n3d_cells: int = 512) -> dict:
    """Heterogeneous batch: n2d_cells x (2D, n=32) then n3d_cells x (3D, n=24)."""
    rng = np.random.default_rng(seed)
    f2 = np.stack([noisy_local_maxwellian(rng, 2, 32, 8.0) for _ in range(n2d_cells)])
    f3 = np.stack([noisy_local_maxwellian(rng, 3, 24, 8.0) for _ in range(n3d_cells)])
    return dict(classes=[dict(d=2, n=32, R=8.0, num_dirs=16, f=f2.astype(np.float32)),
                         dict(d=3, n=24, R=8.0, num_dirs=16, f=f3.astype(np.float32))],
                dt=0.01)


def c5(seed: int = 105, cells: int = 64, n: int = 32) -> dict:
    rng = np.random.default_rng(seed)
    f = np.stack([_three_gaussians(rng, 3, n, 8.0) for _ in range(cells)])
    cot = rng.standard_normal(f.shape)
    return dict(d=3, n=n, R=8.0, num_dirs=16, f=f.astype(np.float32),
                cot=cot.astype(np.float32))


def random_positive(seed: int, d: int, n: int, batch: int = 1) -> np.ndarray:
    """Generic positive test field (i.i.d. U[0.1, 1]) for edge-case tests."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.1, 1.0, size=(batch,) + (n,) * d).astype(np.float32)


def two_maxwellians_batch(seed: int, cells: int, n: int, R: float = 8.0, noise: float = 0.0) -> np.ndarray:
    """`cells` independent draws of the c1/c2 family, shape (cells, n, n), float32.
    Per cell: T1, c1 (2), T2, c2 (2), then the noise field if noise > 0."""
    rng = np.random.default_rng(seed)
    vx, vy = velocity_axes(2, n, R)
    out = np.empty((cells, n, n), dtype=np.float32)
    for c in range(cells):
        f = np.zeros((n, n))
        for _ in range(2):
            T = rng.uniform(0.5, 1.5)
            u = rng.uniform(-2.0, 2.0, size=2)
            f += np.exp(-((vx - u[0]) ** 2 + (vy - u[1]) ** 2) / (2 * T)) / (2 * np.pi * T)
        if noise:
            f *= 1.0 + noise * rng.uniform(-1.0, 1.0, size=f.shape)
        out[c] = f
    return out


def three_gaussians_batch(seed: int, cells: int, n: int, R: float = 8.0) -> np.ndarray:
    """`cells` independent draws of the c3 family, shape (cells, n, n, n), float32."""
    rng = np.random.default_rng(seed)
    return np.stack([_three_gaussians(rng, 3, n, R) for _ in range(cells)]).astype(np.float32)


def relaxation_mix(seed: int, cells: int, d: int, n: int, R: float = 8.0) -> tuple:
    """Spatially inhomogeneous cells at several distances from equilibrium, in
    the order kind = c % 4: a local Maxwellian times (1 + a U[-1,1]) with
    a = 0.002, 0.03 and 0.15, then two unit-mass Maxwellians (T ~ U[0.5, 1.5])
    centred at +-s u, s ~ U[1.5, 2], u a random unit vector (well separated,
    far from equilibrium).  Returns (f of shape (cells,) + (n,) * d, float32;
    kind per cell)."""
    rng = np.random.default_rng(seed)
    out, kind = [], []
    for c in range(cells):
        k = c % 4
        if k < 3:
            out.append(noisy_local_maxwellian(rng, d, n, R, (0.002, 0.03, 0.15)[k]))
        else:
            u = rng.standard_normal(d)
            u *= rng.uniform(1.5, 2.0) / np.linalg.norm(u)
            out.append(maxwellian(d, n, R, 1.0, u, rng.uniform(0.5, 1.5))
                       + maxwellian(d, n, R, 1.0, -u, rng.uniform(0.5, 1.5)))
        kind.append(k)
    return np.stack(out).astype(np.float32), np.array(kind, dtype=np.int32)


def bkw(n: int, R: float, t: float) -> np.ndarray:
    """The BKW solution of the space-homogeneous 2D Maxwell gas (Sec. 4),
    f(t, v) = exp(-|v|^2 / 2S) / (2 pi S^2) (2S - 1 + (1 - S) |v|^2 / (2S)),
    S = 1 - exp(-t/8) / 2, sampled on the n x n grid of [-R, R)^2 (float64).
    Unit mass, zero mean velocity, unit temperature per degree of freedom."""
    vx, vy = velocity_axes(2, n, R)
    v2 = vx * vx + vy * vy
    S = 1.0 - np.exp(-t / 8.0) / 2.0
    return np.exp(-v2 / (2.0 * S)) / (2.0 * np.pi * S * S) * (2.0 * S - 1.0 + (1.0 - S) / (2.0 * S) * v2)
