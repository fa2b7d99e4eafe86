#!/usr/bin/env python3
"""Throughput benchmark of the fast DVM collision operator on one MI355X.

Headline step: one qdvm_eval over a batch of B cells of the 2D workload
(n = 64 points per axis on [-8, 8)^2, Nt = 14, the first 16 lattice lines,
two Maxwellians times (1 + 0.05 xi) per cell).  `value` is cells evaluated
per second (whole job, inputs resident in HBM).  Prints ONE JSON line with
the roofline of the collision kernel (algorithmic FLOPs / measured duration
against the FP32 vector peak), the FP64 oracle timed on the host cores, the
relative error of sampled cells against that oracle, and secondary results:
the other direction counts, 3D n = 32, the batched heterogeneous Euler step
and the adjoint.

    python bench.py [--gpus 1] [--steps 50] [--warmup 5]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Q(f,f) evals/sec, 2D N=64 & 3D N=32 at 1e-5 rel err; % HBM roofline; VJP/eval ratio"
FP32_VECTOR_PEAK_TFLOPS = 157.3      # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2 (packed) x 2.4 GHz
HBM_PEAK_GBS = 8000.0
# sources of the headline kernel k_eval2d<64>: a committed counter summary is used
# only while these files are unchanged since it was taken
KERNEL_SOURCES = ["paper_1201_3986_amd/csrc/kernels_2d.hip", "paper_1201_3986_amd/csrc/cells_2d.h",
                  "paper_1201_3986_amd/csrc/kernels_common.h", "paper_1201_3986_amd/csrc/fft_reg.h",
                  "paper_1201_3986_amd/csrc/qdvm_internal.h"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_flops(dim, n, jobs):
    """Per cell: (P_eff + 1) complex transforms of n^d points at 5 N log2 N, the
    per-direction multiply and product (9 flops per point) and the loss (8)."""
    npts = n ** dim
    return (jobs + 1) * 5.0 * npts * math.log2(npts) + 9.0 * jobs * npts + 8.0 * npts


def vjp_algorithmic_flops(dim, n, jobs):
    npts = n ** dim
    return (2 * jobs + 3) * 5.0 * npts * math.log2(npts) + 20.0 * jobs * npts


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(name):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or None
    when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    s = re.search(r"kernel_source_hash:\s*([0-9a-f]+)", text)
    if not m or not s or s.group(1) != kernel_source_hash():
        return None
    return float(m.group(1))


# algorithmic HBM bytes per cell of each secondary result: f in and Q out
# (8 B per point), plus the second input of the bilinear form and the
# cotangent of the adjoint (12 B per point)
_RESULT_BYTES = {
    "2d_n64_P8": 8 * 4096, "2d_n64_P32": 8 * 4096, "2d_n64_order8": 8 * 4096, "2d_n64_order14": 8 * 4096,
    "2d_n64_P16": 8 * 4096, "2d_n64_P16_near_equilibrium": 8 * 4096, "bilinear_2d_n64_P16": 12 * 4096,
    "vjp_2d_n64_P16": 12 * 4096, "3d_n32_P8": 8 * 32768, "3d_n32_P16": 8 * 32768,
    "bilinear_3d_n32_P16": 12 * 32768, "vjp_3d_n32_P16_64cells": 12 * 32768,
}


def annotate_rooflines(results):
    """Per secondary result: the share of the FP32 vector peak its algorithmic
    FLOPs reach and its algorithmic HBM rate (the bound is the ALU for all)."""
    for key, r in results.items():
        if not isinstance(r, dict):
            continue
        if "tflops" in r:
            r["frac_fp32_peak"] = round(r["tflops"] / FP32_VECTOR_PEAK_TFLOPS, 4)
        if key in _RESULT_BYTES and "cells_per_s" in r:
            gbs = _RESULT_BYTES[key] * r["cells_per_s"] / 1e9
            r["hbm_gbs_algorithmic"] = round(gbs, 1)
            r["hbm_frac_algorithmic"] = round(gbs / HBM_PEAK_GBS, 4)


def platform_info(torch):
    """GPU, HIP and torch versions of the run."""
    info = {"torch": torch.__version__, "hip": getattr(torch.version, "hip", None)}
    try:
        info["gpu"] = torch.cuda.get_device_name(0)
        info["cus"] = torch.cuda.get_device_properties(0).multi_processor_count
    except Exception:  # noqa: BLE001 - informational only
        pass
    try:
        with open("/opt/rocm/.info/version") as fh:
            info["rocm"] = fh.read().strip()
    except OSError:
        pass
    return info


def time_calls(fn, steps, warmup, settle_s=0.15):
    """Average ms per call, HIP events on the current stream (where the library launches).
    settle_s: before the warmup calls, repeat fn for that long, so that a measurement taken
    after a stretch of host work (the GPU idle, its clocks down) starts at settled clocks."""
    import time
    import torch
    t0 = time.time()
    while time.time() - t0 < settle_s:
        fn()
        torch.cuda.synchronize()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def step_percentiles(fn, steps):
    """Per-call durations (ms) with one event pair per call: p10, p50, p90."""
    import torch
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    t = np.array([a.elapsed_time(b) for a, b in evs])
    return [float(np.percentile(t, p)) for p in (10, 50, 90)]


def host_cpu():
    """CPU model and logical CPU count of the host (for the oracle timing)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def cell_errors(plan, f_np, q_np, idx, near_equilibrium_definition=False):
    """Relative L-infinity error of each listed cell against the FP64 oracle
    (Q(f, f); or Q(f, f) - Q(M, M), the near-equilibrium mode's definition)."""
    import oracle
    w = np.float32(plan.weights).astype(np.float64)
    idx = list(idx)
    cells = np.stack([np.asarray(f_np[c], np.float32).astype(np.float64).reshape((plan.n,) * plan.dim)
                      for c in idx])
    if near_equilibrium_definition:
        ref = oracle.collide_near_equilibrium(plan.dim, plan.n, plan.ntilde, plan.dirs, w, cells)
    else:
        ref = oracle.collide(plan.dim, plan.n, plan.ntilde, plan.dirs, w, cells)
    ref = ref.reshape(len(idx), -1)
    got = np.stack([np.asarray(q_np[c], np.float64).reshape(-1) for c in idx])
    return np.max(np.abs(got - ref), axis=1) / np.max(np.abs(ref), axis=1)


def bilinear_errors(plan, g_np, f_np, q_np, idx):
    """Largest relative L-infinity error of the listed cells of Q(g, f) against
    the oracle's pair sum."""
    import oracle
    w = np.float32(plan.weights).astype(np.float64)
    worst = 0.0
    for c in idx:
        ref = oracle.collide_bilinear(plan.dim, plan.n, plan.ntilde, plan.dirs, w,
                                      np.asarray(g_np[c], np.float64), np.asarray(f_np[c], np.float64)).reshape(-1)
        worst = max(worst, float(np.max(np.abs(np.asarray(q_np[c], np.float64).reshape(-1) - ref)) / np.max(np.abs(ref))))
    return worst


def sampled_error(plan, f_np, q_np, idx):
    return float(np.max(cell_errors(plan, f_np, q_np, idx)))


def batched_step(qdvm, workloads, torch, args):
    """The inhomogeneous batch (4096 2D n=32 cells then 512 3D n=24 cells, P = 16):
    one graph-captured Euler step per replay, plain and near-equilibrium, next to
    the same cells through the single-plan kernels (one launch per class)."""
    out = {}
    wl = workloads.c4()
    c2, c3 = wl["classes"]
    f2, f3 = c2["f"].reshape(len(c2["f"]), -1), c3["f"].reshape(len(c3["f"]), -1)
    n2, n3 = len(f2), len(f3)
    flat_np = np.concatenate([f2.reshape(-1), f3.reshape(-1)]).astype(np.float32)
    offs = np.concatenate([np.arange(n2) * 1024, n2 * 1024 + np.arange(n3) * 13824]).astype(np.int64)
    for mode in ("full", "near_equilibrium"):
        p2 = qdvm.Plan(2, 32, 8.0, num_dirs=16, mode=mode)
        p3 = qdvm.Plan(3, 24, 8.0, num_dirs=16, mode=mode)
        b = qdvm.BatchPlan([p2] * n2 + [p3] * n3, offs)
        x = torch.from_numpy(flat_np).cuda()
        s = torch.cuda.Stream()
        g = qdvm.StepGraph(b, x, wl["dt"], s)
        with torch.cuda.stream(s):
            t = time_calls(lambda: g.launch(stream=s), max(5, args.steps // 2), 2)
        y = torch.from_numpy(flat_np).cuda()
        q = torch.empty_like(y)
        y2, y3 = y[:n2 * 1024].view(n2, 1024), y[n2 * 1024:].view(n3, 13824)
        q2, q3 = q[:n2 * 1024].view(n2, 1024), q[n2 * 1024:].view(n3, 13824)

        def single():
            p2.eval(y2, out=q2, dt=wl["dt"])
            p3.eval(y3, out=q3, dt=wl["dt"])
        ts = time_calls(single, max(5, args.steps // 2), 2)
        key = "c4_graph_step" + ("" if mode == "full" else "_near_equilibrium")
        # Q of the initial state (dt = 0) on a seeded sample of cells against the oracle's Q(f, f)
        qd = b.eval(torch.from_numpy(flat_np).cuda())
        qn = qd.cpu().numpy()
        rng = np.random.default_rng(4104)
        s2 = np.sort(rng.choice(n2, size=256, replace=False))
        s3 = np.sort(rng.choice(n3, size=16, replace=False))
        e2 = cell_errors(p2, f2, qn[:n2 * 1024].reshape(n2, -1), s2)
        e3 = cell_errors(p3, f3, qn[n2 * 1024:].reshape(n3, -1), s3)
        rel = float(max(e2.max(), e3.max()))
        out[key] = {"ms": t, "cells_per_s": (n2 + n3) / (t * 1e-3), "tflops": b.flops / (t * 1e-3) / 1e12,
                    "single_plan_launches_ms": ts, "batched_over_single": ts / t,
                    "rel_err_vs_Qff": rel, "rel_err_cells": "256 2D + 16 3D seeded cells",
                    "meets_1e-5": rel <= 1e-5}
        if mode == "full":
            out[key]["note"] = ("plain FP32: gain and loss are 50-100x larger than Q on these near-equilibrium "
                                "cells, so the plain mode does not meet 1e-5; the near-equilibrium step does")
        log("%s: %.3f ms per captured step (%.3e cells/s); single-plan launches %.3f ms; rel err %.2e"
            % (key, t, (n2 + n3) / (t * 1e-3), ts, rel))
        del qd
        g.close()
        b.close()
        p2.close()
        p3.close()
        del x, y, q
    return out


def adaptive_step(qdvm, workloads, torch, args):
    """Adaptive direction count (near-equilibrium plans with P = 4, 8 and 16
    chosen per cell on the device, thresholds 0.004 and 0.04 of the distance
    from the cell's Maxwellian) on cells at four distances from equilibrium
    (workloads.relaxation_mix): 32768 2D n=32 cells and 512 3D n=24 cells,
    each against the same cells all at P = 16 in one batched launch."""
    out = {}
    for d, n, cells, key in ((2, 32, 32768, "adaptive_2d_n32"), (3, 24, 512, "adaptive_3d_n24")):
        f_np, _ = workloads.relaxation_mix(707 + d, min(cells, 4096), d, n)
        f_np = np.ascontiguousarray(np.tile(f_np.reshape(len(f_np), -1), (cells // len(f_np), 1)))
        x = torch.from_numpy(f_np.reshape(-1)).cuda()
        q = torch.empty_like(x)
        offs = np.arange(cells, dtype=np.int64) * n ** d
        plans = [qdvm.Plan(d, n, 8.0, num_dirs=P, mode="near_equilibrium") for P in (4, 8, 16)]
        ad = qdvm.AdaptivePlan(plans, offs, [0.004, 0.04])
        _, lv, _ = ad.eval(x, out=q, levels=True)
        counts = np.bincount(lv.cpu().numpy(), minlength=3)
        ta = time_calls(lambda: ad.eval(x, out=q), max(5, args.steps // 2), 2)
        b = qdvm.BatchPlan([plans[2]] * cells, offs)
        tu = time_calls(lambda: b.eval(x, out=q), max(5, args.steps // 2), 2)
        log("%s: P in (4, 8, 16), near-equilibrium mode, %d cells (per level %s): %.3f ms; all at P=16 %.3f ms"
            % (key, cells, counts.tolist(), ta, tu))
        out[key] = {"ms": ta, "cells_per_s": cells / (ta * 1e-3), "cells_per_level_P4_P8_P16": counts.tolist(),
                    "uniform_P16_ms": tu, "speedup_vs_uniform_P16": tu / ta}
        ad.close()
        b.close()
        for p in plans:
            p.close()
        del x, q
    return out


def transform_choice(qdvm, workloads, torch, args):
    """The transform stage at 2D n = 16 (262144 cells), the register FFT of the
    collision kernels against the DFT as FP32 matrix-core products: one forward
    transform per cell (I/O bound) and 17 (8 inverse-forward round trips in
    registers, as compute-bound as the fused evaluation); and the O(n^4)
    pseudo-spectral FP64 form against the fast path on 1024 cells."""
    out = {}
    B = 1 << 18
    base = workloads.two_maxwellians_batch(4300, 256, 16, noise=0.05)
    f = torch.from_numpy(np.ascontiguousarray(np.tile(base, (B // 256, 1, 1)))).cuda()
    st = {}
    for m, name in ((0, "register_fft"), (1, "mfma_dft")):
        for reps in (0, 8):
            t = time_calls(lambda: qdvm.transform_stage(f, m, reps), max(5, args.steps // 5), 2)
            st["%s_transforms_%d_ms" % (name, 2 * reps + 1)] = t
    per_fft = (st["register_fft_transforms_17_ms"] - st["register_fft_transforms_1_ms"]) / 16
    per_mfma = (st["mfma_dft_transforms_17_ms"] - st["mfma_dft_transforms_1_ms"]) / 16
    st.update({"cells": B, "ms_per_transform_register_fft": per_fft, "ms_per_transform_mfma_dft": per_mfma,
               "mfma_over_fft": per_mfma / per_fft})
    out["transform_stage_2d_n16"] = st
    log("transform stage 2D n=16, %d cells: FFT %.4f ms, MFMA DFT %.4f ms per transform (x%.2f)"
        % (B, per_fft, per_mfma, per_mfma / per_fft))
    pl = qdvm.Plan(2, 16, 8.0, farey_order=4)
    g = f[:1024].contiguous()
    tp = time_calls(lambda: pl.eval_pseudo_spectral(g), 3, 1)
    tf = time_calls(lambda: pl.eval(g), 10, 2)
    out["pseudo_spectral_2d_n16_order4"] = {"cells": 1024, "ms": tp, "fast_path_ms": tf, "ratio": tp / tf,
                                            "note": "O(n^4) FP64 direct sums (Sec. 3.1) vs the O(P n^2 log n) FP32 path"}
    log("pseudo-spectral 2D n=16 order 4, 1024 cells: %.3f ms (fast path %.4f ms)" % (tp, tf))
    pl.close()
    return out


def profile_workload(args, qdvm, workloads, torch):
    """One secondary workload alone: 3D n=32 P=16 on 2048 cells, its adjoint on
    the 64-cell differentiation batch, the adjoint and the near-equilibrium
    mode on 16384 2D n=64 cells, or the captured batched Euler step."""
    if args.profile_workload == "3d_n32_p16":
        base3 = workloads.three_gaussians_batch(303, 64, 32)
        f3 = torch.from_numpy(np.ascontiguousarray(np.tile(base3, (32, 1, 1, 1)))).cuda()
        q3 = torch.empty_like(f3)
        pl = qdvm.Plan(3, 32, 8.0, num_dirs=16)
        t = time_calls(lambda: pl.eval(f3, out=q3), args.steps, args.warmup, settle_s=0.0)
        print(json.dumps({"workload": "3D n=32 P=16, 2048 cells", "ms": t}), flush=True)
    elif args.profile_workload == "vjp_3d_n32_p16":
        c5 = workloads.c5()
        fv = torch.from_numpy(c5["f"]).cuda()
        cv = torch.from_numpy(c5["cot"]).cuda()
        pl = qdvm.Plan(3, 32, 8.0, num_dirs=16)
        t = time_calls(lambda: pl.vjp(fv, cv), args.steps, args.warmup, settle_s=0.0)
        print(json.dumps({"workload": "adjoint 3D n=32 P=16, 64 cells", "ms": t}), flush=True)
    elif args.profile_workload == "vjp_2d_n64_p16":
        base = workloads.two_maxwellians_batch(202, 64, 64, noise=0.05)
        f = torch.from_numpy(np.ascontiguousarray(np.tile(base, (256, 1, 1)))).cuda()
        cot = torch.from_numpy(np.random.default_rng(106).standard_normal(f.shape).astype(np.float32)).cuda()
        pl = qdvm.Plan(2, 64, 8.0, num_dirs=16)
        t = time_calls(lambda: pl.vjp(f, cot), args.steps, args.warmup, settle_s=0.0)
        print(json.dumps({"workload": "adjoint 2D n=64 P=16, 16384 cells", "ms": t}), flush=True)
    elif args.profile_workload == "near_2d_n64_p16":
        base = workloads.two_maxwellians_batch(202, 64, 64, noise=0.05)
        f = torch.from_numpy(np.ascontiguousarray(np.tile(base, (256, 1, 1)))).cuda()
        q = torch.empty_like(f)
        pl = qdvm.Plan(2, 64, 8.0, num_dirs=16, mode="near_equilibrium")
        t = time_calls(lambda: pl.eval(f, out=q), args.steps, args.warmup, settle_s=0.0)
        print(json.dumps({"workload": "near-equilibrium 2D n=64 P=16, 16384 cells", "ms": t}), flush=True)
    else:
        r = batched_step(qdvm, workloads, torch, args)
        print(json.dumps({"workload": "batched Euler step, 4096 2D n=32 + 512 3D n=24 cells", "results": r}),
              flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--batch", type=int, default=16384, help="2D n=64 cells per step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB elementwise copy (x*1 -> y) to scale HBM counters")
    ap.add_argument("--profile-workload",
                    choices=["3d_n32_p16", "vjp_3d_n32_p16", "vjp_2d_n64_p16", "near_2d_n64_p16", "c4_step"],
                    default=None,
                    help="run only this secondary workload's timed loop (for counter collection) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(cells shard across GPUs without communication; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1201_3986_amd import qdvm, workloads

    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    qdvm.load()
    results = {}

    if args.profile_workload:
        profile_workload(args, qdvm, workloads, torch)
        return

    # ---------------------------------------------------------------- headline
    B = args.batch
    distinct = 256
    base = workloads.two_maxwellians_batch(202, distinct, 64, noise=0.05)
    f_np = np.ascontiguousarray(np.tile(base, (B // distinct + 1, 1, 1))[:B])
    f = torch.from_numpy(f_np).cuda()
    q = torch.empty_like(f)
    plan = qdvm.Plan(2, 64, 8.0, num_dirs=16)
    log("headline: 2D n=64 P=16 jobs=%d batch=%d" % (plan.num_jobs, B))
    ms = time_calls(lambda: plan.eval(f, out=q), args.steps, args.warmup, settle_s=0.0)
    pct = step_percentiles(lambda: plan.eval(f, out=q), min(args.steps, 50))
    value = B / (ms * 1e-3)
    flops = algorithmic_flops(2, 64, plan.num_jobs) * B
    achieved = flops / (ms * 1e-3) / 1e12
    q_np = q.cpu().numpy()
    # every distinct cell of the step against the oracle (the batch tiles 256 draws)
    n_check = min(distinct, B)
    head_errs = cell_errors(plan, f_np, q_np, range(n_check))
    err = float(head_errs.max())
    tiles_equal = all(np.array_equal(q_np[:n_check], q_np[t:t + n_check])
                      for t in range(n_check, B - n_check + 1, n_check))
    log("headline: %.3f ms/step, %.3e cells/s, %.1f TFLOP/s, rel err over %d distinct cells %.2e (cell %d)"
        % (ms, value, achieved, n_check, err, int(np.argmax(head_errs))))
    traffic = recorded_traffic("eval2d_n64_p16_traffic.md")
    roofline = {
        "bound": "alu", "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
        "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
        "traffic": (traffic * 1.0) if traffic is not None else None,
        "kernel": "k_eval2d<64, 0, false, true> (per-job multiplier tables; one launch per step)",
        "note": "FP32 vector peak counts packed (2-wide) FMA; this code is built without packed FP32 "
                "instructions, so its own issue ceiling is half of it (78.6 TFLOP/s)",
        "algorithmic_flops_per_cell": algorithmic_flops(2, 64, plan.num_jobs),
        "hbm_gbs_algorithmic": round(8.0 * 4096 * B / (ms * 1e-3) / 1e9, 1),
        "hbm_frac_algorithmic": round(8.0 * 4096 * B / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
    }

    if args.copy_calibration:
        x = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        log("copy calibration: 3 x (read 256 MiB, write 256 MiB) elementwise kernels")
        del x, y

    # ---------------------------------------------------------------- secondary
    if not args.no_secondary:
        for P in (8, 32):
            pl = qdvm.Plan(2, 64, 8.0, num_dirs=P)
            t = time_calls(lambda: pl.eval(f, out=q), max(5, args.steps // 4), 2)
            e = sampled_error(pl, f_np, q.cpu().numpy(), range(n_check))
            results["2d_n64_P%d" % P] = {"cells_per_s": B / (t * 1e-3), "ms": t, "rel_err": e,
                                         "rel_err_cells": n_check,
                                         "tflops": algorithmic_flops(2, 64, pl.num_jobs) * B / (t * 1e-3) / 1e12}
            pl.close()
        # the whole line sets of Farey order 8 (88 lines) and 14 (every line of the
        # box at Nt = 14: 256 lines), the two extra points of the 2D n = 64 sweep
        for order in (8, 14):
            pl = qdvm.Plan(2, 64, 8.0, farey_order=order)
            t = time_calls(lambda: pl.eval(f, out=q), 5, 1)
            e = sampled_error(pl, f_np, q.cpu().numpy(), range(n_check))
            results["2d_n64_order%d" % order] = {
                "lines": pl.num_dirs, "cells_per_s": B / (t * 1e-3), "ms": t, "rel_err": e,
                "rel_err_cells": n_check, "meets_1e-5": e <= 1e-5,
                "note": "whole line set, not a configuration of the sweep; FP32 limit on the cells whose gain "
                        "and loss are ~33 max|Q| at the peak",
                "tflops": algorithmic_flops(2, 64, pl.num_jobs) * B / (t * 1e-3) / 1e12}
            log("2D n=64 Farey order %d (%d lines): %.3f ms, rel err %.2e" % (order, pl.num_dirs, t, e))
            pl.close()
        results["2d_n64_P16"] = {"cells_per_s": value, "ms": ms, "rel_err": err, "rel_err_cells": n_check,
                                 "tflops": achieved}
        # PCIe-inclusive rate: f from pinned host memory, Q back to pinned host memory
        fh = torch.empty(f.shape, dtype=torch.float32, pin_memory=True)
        fh.copy_(torch.from_numpy(f_np))
        qh = torch.empty_like(fh, pin_memory=True)

        def with_pcie():
            f.copy_(fh, non_blocking=True)
            plan.eval(f, out=q)
            qh.copy_(q, non_blocking=True)
        t = time_calls(with_pcie, max(5, args.steps // 4), 2)
        results["2d_n64_P16_pcie_inclusive"] = {"cells_per_s": B / (t * 1e-3), "ms": t,
                                                "note": "host f -> device, eval, Q -> host, one stream"}
        log("PCIe-inclusive 2D n=64 P=16: %.3f ms (%.3e cells/s)" % (t, B / (t * 1e-3)))
        del fh, qh
        # the same cells in the near-equilibrium mode (rel err against the oracle's Q(f, f))
        pn = qdvm.Plan(2, 64, 8.0, num_dirs=16, mode="near_equilibrium")
        t = time_calls(lambda: pn.eval(f, out=q), max(5, args.steps // 4), 2)
        qn = q.cpu().numpy()
        e_ff = cell_errors(pn, f_np, qn, range(n_check))
        e_def = cell_errors(pn, f_np, qn, range(n_check), near_equilibrium_definition=True)
        results["2d_n64_P16_near_equilibrium"] = {
            "cells_per_s": B / (t * 1e-3), "ms": t, "rel_err_vs_definition": float(e_def.max()),
            "rel_err_vs_Qff": float(e_ff.max()), "cells_checked": n_check,
            "note": "the mode returns Q(f,f) - Q(M,M); on these two-Maxwellian cells the fitted M is wide and "
                    "its periodic-wrap residue Q(M,M) is not negligible, so it is not an evaluation of Q(f,f) here"}
        log("near-equilibrium 2D n=64 P=16: %.3f ms, rel err vs definition %.2e, vs Q(f,f) %.2e"
            % (t, e_def.max(), e_ff.max()))
        pn.close()
        # bilinear Q(g, f) on the headline cells, g = the cells shifted by one
        gsh = torch.roll(f, 1, dims=0).contiguous()
        tb = time_calls(lambda: plan.eval_bilinear(gsh, f, out=q), max(5, args.steps // 4), 2)
        eb = bilinear_errors(plan, np.roll(f_np, 1, axis=0), f_np, q.cpu().numpy(), range(0, n_check, 32))
        results["bilinear_2d_n64_P16"] = {
            "ms": tb, "cells_per_s": B / (tb * 1e-3), "eval_ms_same_batch": ms, "bilinear_over_eval": tb / ms,
            "rel_err": eb, "rel_err_cells": len(range(0, n_check, 32)),
            "note": "Q(g, f) with g the cells shifted by one: 2 forward + 1 loss + P inverse transforms per cell"}
        log("bilinear Q(g,f) 2D n=64 P=16: %.3f ms (eval %.3f ms), rel err %.2e" % (tb, ms, eb))
        del gsh
        # 2D adjoint on the headline cells (same f, a N(0,1) cotangent)
        cot = torch.from_numpy(np.random.default_rng(106).standard_normal(f.shape).astype(np.float32)).cuda()
        tv = time_calls(lambda: plan.vjp(f, cot), max(5, args.steps // 5), 2)
        results["vjp_2d_n64_P16"] = {
            "ms": tv, "eval_ms_same_batch": ms, "vjp_over_eval": tv / ms, "cells_per_s": B / (tv * 1e-3),
            "tflops": vjp_algorithmic_flops(2, 64, plan.num_jobs) * B / (tv * 1e-3) / 1e12}
        log("VJP 2D n=64 P=16 %d cells: %.3f ms (eval %.3f ms, ratio %.2f)" % (B, tv, ms, tv / ms))
        del cot
        del f, q
        torch.cuda.empty_cache()

        C3 = 2048
        base3 = workloads.three_gaussians_batch(303, 64, 32)
        f3_np = np.ascontiguousarray(np.tile(base3, (C3 // 64, 1, 1, 1)))
        f3 = torch.from_numpy(f3_np).cuda()
        q3 = torch.empty_like(f3)
        ev3 = {}
        for P in (8, 16):
            pl = qdvm.Plan(3, 32, 8.0, num_dirs=P)
            t = time_calls(lambda: pl.eval(f3, out=q3), max(5, args.steps // 5), 2)
            e = sampled_error(pl, f3_np, q3.cpu().numpy(), [1, 22, 45, 63])
            ev3[P] = t
            results["3d_n32_P%d" % P] = {"cells_per_s": C3 / (t * 1e-3), "ms": t, "rel_err": e,
                                         "rel_err_cells": 4,
                                         "tflops": algorithmic_flops(3, 32, pl.num_jobs) * C3 / (t * 1e-3) / 1e12}
            log("3D n=32 P=%d: %.3f ms for %d cells, rel err %.2e" % (P, t, C3, e))
            if P == 16:
                g3 = torch.roll(f3, 1, dims=0).contiguous()
                tb = time_calls(lambda: pl.eval_bilinear(g3, f3, out=q3), max(5, args.steps // 5), 2)
                eb = bilinear_errors(pl, np.roll(f3_np, 1, axis=0), f3_np, q3.cpu().numpy(), [1, 40])
                results["bilinear_3d_n32_P16"] = {"ms": tb, "cells_per_s": C3 / (tb * 1e-3), "eval_ms_same_batch": t,
                                                  "bilinear_over_eval": tb / t, "rel_err": eb, "rel_err_cells": 2}
                log("bilinear Q(g,f) 3D n=32 P=16: %.3f ms (eval %.3f ms), rel err %.2e" % (tb, t, eb))
                del g3
            if P == 16:
                # adjoint on the differentiation workload shape (64 cells, P = 16)
                c5 = workloads.c5()
                fv = torch.from_numpy(c5["f"]).cuda()
                cv = torch.from_numpy(c5["cot"]).cuda()
                tv = time_calls(lambda: pl.vjp(fv, cv), max(5, args.steps // 5), 2)
                te = time_calls(lambda: pl.eval(fv), max(5, args.steps // 5), 2)
                results["vjp_3d_n32_P16_64cells"] = {
                    "ms": tv, "eval_ms_same_batch": te, "vjp_over_eval": tv / te,
                    "cells_per_s": 64 / (tv * 1e-3),
                    "tflops": vjp_algorithmic_flops(3, 32, pl.num_jobs) * 64 / (tv * 1e-3) / 1e12}
                log("VJP 3D n=32 P=16 64 cells: %.3f ms (eval %.3f ms, ratio %.2f)" % (tv, te, tv / te))
            pl.close()
        del f3, q3
        torch.cuda.empty_cache()
        results.update(transform_choice(qdvm, workloads, torch, args))
        results.update(batched_step(qdvm, workloads, torch, args))
        results.update(adaptive_step(qdvm, workloads, torch, args))

    # ---------------------------------------------------------------- CPU oracle
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        threads = oracle.num_threads()
        w = np.float32(plan.weights).astype(np.float64)
        cells = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < 12.0 and cells < B:
            oracle.collide(2, 64, plan.ntilde, plan.dirs, w, f_np[cells % distinct].astype(np.float64))
            cells += 1
        dt = time.perf_counter() - t0
        cpu = {"value": cells / dt, "unit": "evals/s", "cores": threads, "kind": "oracle",
               "sample": "%d cells of the headline workload (2D n=64, P=16), FP64 direct pair sum, "
                         "%.1f s wall, OpenMP threads=%d" % (cells, dt, threads),
               "host": host_cpu()}
        log("cpu oracle: %.2f cells/s on %d threads" % (cells / dt, threads))

    annotate_rooflines(results)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2D DVM n=64 on [-8,8)^2, Nt=14, first 16 lattice lines (8 perpendicular "
                               "pairs), two Maxwellians x (1 + 0.05 U[-1,1]) per cell, %d cells per step" % B,
                   "dim": 2, "n": 64, "half_width": 8.0, "ntilde": plan.ntilde, "num_dirs": 16,
                   "cells_per_step": B, "parallelism": "single GPU"},
        "step_ms_p10_p50_p90": pct,
        "parity": {"rel_linf": err, "cells_checked": n_check, "distinct_cells_in_step": n_check,
                   "median_cell_rel_linf": float(np.median(head_errs)), "tolerance": 1e-5,
                   "meets_tolerance": err <= 1e-5, "tiles_bit_identical": bool(tiles_equal)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "results": results,
        "platform": platform_info(torch),
    }
    plan.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
