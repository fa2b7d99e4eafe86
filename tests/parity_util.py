"""Shared helpers of the GPU parity tests: run the oracle on exactly the inputs
the GPU saw (FP32 values promoted to FP64, the plan's weights rounded to FP32)
and measure the relative L-infinity error."""
import numpy as np

import oracle


def oracle_q(plan, f32, w=None):
    """Oracle Q for the cells of f32 (numpy float32, batch * n^d) under `plan`."""
    weights = np.float32(plan.weights if w is None else w).astype(np.float64)
    f64 = np.asarray(f32, dtype=np.float32).astype(np.float64)
    return oracle.collide(plan.dim, plan.n, plan.ntilde, plan.dirs, weights, f64)


def oracle_vjp(plan, f32, c32, w=None):
    weights = np.float32(plan.weights if w is None else w).astype(np.float64)
    return oracle.vjp(plan.dim, plan.n, plan.ntilde, plan.dirs, weights,
                      np.asarray(f32, np.float32).astype(np.float64),
                      np.asarray(c32, np.float32).astype(np.float64))


def rel_linf(got, ref, scale=None):
    got = np.asarray(got, dtype=np.float64).reshape(-1)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1)
    s = float(np.max(np.abs(ref))) if scale is None else float(scale)
    return float(np.max(np.abs(got - ref))) / s


def per_cell_rel_linf(got, ref, npts):
    got = np.asarray(got, np.float64).reshape(-1, npts)
    ref = np.asarray(ref, np.float64).reshape(-1, npts)
    return np.max(np.abs(got - ref), axis=1) / np.max(np.abs(ref), axis=1)


def loss_total(plan, f):
    """sum_i f_i l_i, l = sum_p w_p (line * plane convolution of f), via numpy FFTs."""
    n, d = plan.n, plan.dim
    f = np.asarray(f, np.float64).reshape((n,) * d)
    F = np.fft.fftn(f)
    tot = np.zeros_like(f)
    import itertools
    box = list(itertools.product(range(-plan.ntilde, plan.ntilde + 1), repeat=d))
    for e, w, M in zip(plan.dirs, np.float32(plan.weights).astype(np.float64), plan.line_len):
        if M == 0:
            continue
        IK = np.zeros(f.shape)
        for m in range(-M, M + 1):
            if m:
                IK[tuple((m * e) % n)] += 1.0
        IL = np.zeros(f.shape)
        for l in box:
            if int(np.dot(l, e)) == 0:
                IL[tuple(np.array(l) % n)] += 1.0
        tot += w * np.fft.ifftn(F * np.fft.fftn(IK) * np.fft.fftn(IL)).real
    return float(np.sum(f * tot))
