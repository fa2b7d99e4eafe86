"""Shared helpers of the GPU parity tests: run the oracle on exactly the inputs
the GPU saw (FP32 values promoted to FP64, the plan's weights rounded to FP32)
and measure the relative L-infinity error."""
import numpy as np

import oracle


def assert_oracle_direction_set(plan):
    """The set a GPU test checks must be the oracle's own: where the plan took
    the library's defaults (first P lines, every line of a Farey order, default
    weights, default Nt), its lists must equal the oracle's enumeration, so a
    regression in the product's plan builder cannot pass a parity test by
    handing the oracle the same wrong set."""
    r = getattr(plan, "request", None)
    assert r is not None, "plan without its request record"
    if r["ntilde"] == 0:
        assert plan.ntilde == oracle.default_ntilde(plan.n), (plan.ntilde, plan.n)
    if not r["explicit_dirs"]:
        ref = oracle.first_lines(plan.dim, r["num_dirs"]) if r["num_dirs"] > 0 \
            else oracle.lines(plan.dim, r["farey_order"])
        assert np.array_equal(np.asarray(plan.dirs), ref), "plan directions differ from the oracle's"
    if not r["explicit_weights"]:
        h = 2.0 * r["half_width"] / plan.n
        ref_w = oracle.default_weights(plan.dim, h, plan.dirs, getattr(plan, "line_weight", 0))
        assert np.allclose(plan.weights, ref_w, rtol=1e-14, atol=0.0), "plan weights differ from the oracle's"


def oracle_q(plan, f32, w=None):
    """Oracle Q for the cells of f32 (numpy float32, batch * n^d) under `plan`."""
    assert_oracle_direction_set(plan)
    weights = np.float32(plan.weights if w is None else w).astype(np.float64)
    f64 = np.asarray(f32, dtype=np.float32).astype(np.float64)
    return oracle.collide(plan.dim, plan.n, plan.ntilde, plan.dirs, weights, f64, getattr(plan, "line_weight", 0))


def oracle_vjp(plan, f32, c32, w=None):
    assert_oracle_direction_set(plan)
    weights = np.float32(plan.weights if w is None else w).astype(np.float64)
    return oracle.vjp(plan.dim, plan.n, plan.ntilde, plan.dirs, weights,
                      np.asarray(f32, np.float32).astype(np.float64),
                      np.asarray(c32, np.float32).astype(np.float64), getattr(plan, "line_weight", 0))


def oracle_grad_w(plan, f32, c32):
    """grad_w of <c, Q(f; w)> summed over the cells: Q is linear in w, so
    grad_w[p] = sum_cells <c, Q_p> with Q_p the oracle's unit-weight term of
    direction p (its direct pair sum)."""
    assert_oracle_direction_set(plan)
    f = np.asarray(f32, np.float32).astype(np.float64).reshape(-1, plan.npts)
    c = np.asarray(c32, np.float32).astype(np.float64).reshape(-1, plan.npts)
    gw = np.zeros(plan.num_dirs)
    for k in range(f.shape[0]):
        terms = oracle.collide_terms(plan.dim, plan.n, plan.ntilde, plan.dirs, f[k], getattr(plan, "line_weight", 0))
        gw += terms @ c[k]
    return gw


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
