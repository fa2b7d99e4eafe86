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
