"""GPU heterogeneous batch (one persistent launch per block-size family) and
the graph-captured Euler step.

* batched results equal the single-cell path bit for bit (same device code,
  same multipliers) and the FP64 oracle on sampled cells (<= 1e-5 of max|Q|);
* mixed grid sizes, plans and ragged work items; in-place Euler updates;
* the captured step is replayed several times with eager work between the
  replays, and every replay is checked against the eager result.
"""
import numpy as np
import pytest

from paper_1201_3986_amd import workloads
from parity_util import loss_total, oracle_q, per_cell_rel_linf, rel_linf

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def assert_same_cell(plan, got, single):
    """The batched launch runs the single-cell device code, so 2D cells with
    n < 32 match the single-plan result bit for bit.  Three cases agree to
    rounding only: a small 3D batch through the single-plan path spreads each
    cell's directions over several workgroups and adds their parts in another
    order; a single near-equilibrium 2D n = 64 plan runs the two-wave kernel,
    which splits each job's gain over two accumulators; and a single plain 2D
    plan at n = 64 (and at n = 32 for large batches) folds the job weights into
    per-job multiplier tables (the weight enters as two square-root factors
    instead of one product)."""
    got = np.asarray(got).reshape(-1)
    single = np.asarray(single).reshape(-1)
    if plan.dim == 2 and plan.n < 32:
        assert np.array_equal(got, single)
    else:
        assert rel_linf(got, single) <= 1e-6


def c4_sample(n2, n3, k2=256, k3=64):
    """Seeded sample of the batched workload's cells checked against the oracle:
    256 of the 2D cells and 64 of the 3D cells (sorted indices)."""
    rng = np.random.default_rng(4104)
    return np.sort(rng.choice(n2, size=k2, replace=False)), np.sort(rng.choice(n3, size=k3, replace=False))


def _layout(cells):
    """cells: list of (plan, array) -> flat f, offsets (with gaps between cells)."""
    offs, pos = [], 0
    for plan, a in cells:
        offs.append(pos)
        pos += plan.npts + 37            # gaps: offsets need not be packed
    flat = np.full(pos, -7.0, dtype=np.float32)
    for (plan, a), o in zip(cells, offs):
        flat[o:o + plan.npts] = a.reshape(-1)
    return flat, np.array(offs, dtype=np.int64)


def test_mixed_batch_equals_single_cell_and_oracle(gpu_lib):
    import torch
    p32 = gpu_lib.Plan(2, 32, 8.0, num_dirs=16)
    p32b = gpu_lib.Plan(2, 32, 8.0, num_dirs=7)
    p16 = gpu_lib.Plan(2, 16, 8.0, farey_order=4)
    p24 = gpu_lib.Plan(3, 24, 8.0, num_dirs=16)
    rng = np.random.default_rng(4)
    cells = []
    for i in range(45):           # 2D n=32: items of 8 cells and ragged tails, two plans interleaved
        cells.append((p32 if i % 3 else p32b, workloads.random_positive(500 + i, 2, 32)[0]))
    for i in range(3):
        cells.append((p24, workloads.random_positive(600 + i, 3, 24)[0]))
    for i in range(40):           # 2D n=16: 16 cells per item
        cells.append((p16, workloads.random_positive(700 + i, 2, 16)[0]))
    order = rng.permutation(len(cells))
    cells = [cells[k] for k in order]
    flat, offs = _layout(cells)
    b = gpu_lib.BatchPlan([c[0] for c in cells], offs)
    # 256-thread family (2D; items of uneven cost, so its queue counter is
    # reset by a kernel first) and 576-thread family (3D n=24, even items)
    assert b.launches == 3
    fd = _dev(flat)
    qd = b.eval(fd)
    torch.cuda.synchronize()
    q = qd.cpu().numpy()
    for k, ((plan, a), o) in enumerate(zip(cells, offs)):
        single = plan.eval(_dev(a))
        torch.cuda.synchronize()
        assert_same_cell(plan, q[o:o + plan.npts], single.cpu().numpy())
    for k in (0, 7, len(cells) - 1):
        plan, a = cells[k]
        o = offs[k]
        err = rel_linf(q[o:o + plan.npts], oracle_q(plan, a))
        assert err <= TOL, (k, err)


def test_two_families_and_in_place_euler(gpu_lib):
    import torch
    p64 = gpu_lib.Plan(2, 64, 8.0, num_dirs=16)
    p32 = gpu_lib.Plan(3, 32, 8.0, num_dirs=8)
    p8 = gpu_lib.Plan(2, 8, 4.0, ntilde=2, num_dirs=4)
    cells = [(p64, workloads.random_positive(800 + i, 2, 64)[0]) for i in range(11)]
    cells += [(p32, workloads.random_positive(900 + i, 3, 32)[0]) for i in range(2)]
    cells += [(p8, workloads.random_positive(950 + i, 2, 8)[0]) for i in range(5)]
    flat, offs = _layout(cells)
    b = gpu_lib.BatchPlan([c[0] for c in cells], offs)
    # 512-thread family (2D n=64 items of 8 and 3 cells: uneven, counter reset
    # first) and 256-thread family (one 2D n=8 item)
    assert b.launches == 3
    dt = 0.01
    x = _dev(flat)
    b.eval(x, out=x, dt=dt)
    torch.cuda.synchronize()
    got = x.cpu().numpy()
    for (plan, a), o in zip(cells, offs):
        ref = plan.eval(_dev(a), dt=dt)
        torch.cuda.synchronize()
        assert_same_cell(plan, got[o:o + plan.npts], ref.cpu().numpy())
    # gaps between cells untouched
    mask = np.ones(len(flat), bool)
    for (plan, a), o in zip(cells, offs):
        mask[o:o + plan.npts] = False
    assert np.all(got[mask] == -7.0)


def test_unsupported_and_invalid(gpu_lib):
    p16 = gpu_lib.Plan(3, 16, 8.0, num_dirs=8)
    with pytest.raises(gpu_lib.QdvmError) as ei:
        gpu_lib.BatchPlan([p16], [0])
    assert ei.value.status == gpu_lib.QDVM_EUNSUPPORTED
    p = gpu_lib.Plan(2, 32, 8.0, num_dirs=8)
    with pytest.raises(gpu_lib.QdvmError) as ei:
        gpu_lib.BatchPlan([p], [-5])
    assert ei.value.status == gpu_lib.QDVM_EINVAL


def test_config4_graph_step(gpu_lib):
    """The batched inhomogeneous workload: 4096 2D n=32 cells then 512 3D n=24
    cells, P = 16, one captured forward-Euler step with dt = 0.01."""
    import torch
    wl = workloads.c4()
    c2, c3 = wl["classes"]
    p2 = gpu_lib.Plan(2, 32, 8.0, num_dirs=16)
    p3 = gpu_lib.Plan(3, 24, 8.0, num_dirs=16)
    f2, f3 = c2["f"].reshape(len(c2["f"]), -1), c3["f"].reshape(len(c3["f"]), -1)
    plans = [p2] * len(f2) + [p3] * len(f3)
    offs = np.concatenate([np.arange(len(f2)) * 1024, len(f2) * 1024 + np.arange(len(f3)) * 13824]).astype(np.int64)
    flat = np.concatenate([f2.reshape(-1), f3.reshape(-1)]).astype(np.float32)
    b = gpu_lib.BatchPlan(plans, offs)
    assert b.launches == 2        # even items in both families: no counter resets
    dt = wl["dt"]
    # eager reference trajectory
    ref = _dev(flat)
    eager = []
    for _ in range(3):
        b.eval(ref, out=ref, dt=dt)
        torch.cuda.synchronize()
        eager.append(ref.cpu().numpy())
    # graph on a side stream, replayed with eager work and synchronisation between replays
    x = _dev(flat)
    s = torch.cuda.Stream()
    g = gpu_lib.StepGraph(b, x, dt, s)
    for k in range(3):
        g.launch(stream=s)
        s.synchronize()
        scratch = torch.ones(1 << 20, device="cuda") * 3.0       # unrelated eager work
        torch.cuda.synchronize()
        assert np.array_equal(x.cpu().numpy(), eager[k]), k
        del scratch
    # physics of one step: mass per cell, positivity, and Q against the oracle
    q = b.eval(_dev(flat))
    torch.cuda.synchronize()
    qn = q.cpu().numpy()
    step1 = eager[0]
    # Prop. 3.3: the step keeps f >= 0 when dt * (loss frequency) < 1; in FP32
    # the tails may dip below zero by at most the rounding of dt * Q
    print("config4: min after one step %.3e, max f %.3e" % (np.min(step1), np.max(flat)))
    assert np.min(step1) >= -dt * TOL * np.max(np.abs(qn))
    # mass residual per cell relative to the total loss it balances (sum_i f_i l_i)
    worst_mass = 0.0
    for i in range(len(plans)):
        o, n = offs[i], plans[i].npts
        qi = qn[o:o + n].astype(np.float64)
        worst_mass = max(worst_mass, abs(qi.sum()) / loss_total(plans[i], flat[o:o + n]))
    print("config4: worst per-cell mass residual (relative to the loss) %.3e" % worst_mass)
    s2, s3 = c4_sample(len(f2), len(f3))
    e2 = per_cell_rel_linf(qn[:len(f2) * 1024].reshape(len(f2), -1)[s2], oracle_q(p2, f2[s2]), 1024)
    e3 = per_cell_rel_linf(qn[len(f2) * 1024:].reshape(len(f3), -1)[s3], oracle_q(p3, f3[s3]), 13824)
    print("config4 plain FP32: %d 2D cells max rel err %.2e (%d above 1e-5), %d 3D cells max %.2e (%d above)"
          % (len(s2), e2.max(), int(np.sum(e2 > TOL)), len(s3), e3.max(), int(np.sum(e3 > TOL))))
    assert worst_mass <= 1e-6
    # plain FP32 does not reach 1e-5 of max|Q| on these near-equilibrium cells
    # (gain and loss are 50-100x larger than Q); the near-equilibrium mode does
    # (next test).  Here the plain mode is held to its documented bound.
    assert max(e2.max(), e3.max()) <= 1e-4


def test_config4_graph_step_near_equilibrium(gpu_lib):
    """The batched inhomogeneous workload in the near-equilibrium mode: every
    sampled cell within 1e-5 of max|Q| of the oracle's Q(f, f), replays equal
    to the eager step, and plain and near-equilibrium plans mixed in one batch
    give the single-plan results bit for bit."""
    import torch
    import oracle
    wl = workloads.c4()
    c2, c3 = wl["classes"]
    near = "near_equilibrium"
    p2 = gpu_lib.Plan(2, 32, 8.0, num_dirs=16, mode=near)
    p3 = gpu_lib.Plan(3, 24, 8.0, num_dirs=16, mode=near)
    f2, f3 = c2["f"].reshape(len(c2["f"]), -1), c3["f"].reshape(len(c3["f"]), -1)
    plans = [p2] * len(f2) + [p3] * len(f3)
    offs = np.concatenate([np.arange(len(f2)) * 1024, len(f2) * 1024 + np.arange(len(f3)) * 13824]).astype(np.int64)
    flat = np.concatenate([f2.reshape(-1), f3.reshape(-1)]).astype(np.float32)
    b = gpu_lib.BatchPlan(plans, offs)
    dt = wl["dt"]
    ref = _dev(flat)
    eager = []
    for _ in range(2):
        b.eval(ref, out=ref, dt=dt)
        torch.cuda.synchronize()
        eager.append(ref.cpu().numpy())
    x = _dev(flat)
    s = torch.cuda.Stream()
    g = gpu_lib.StepGraph(b, x, dt, s)
    for k in range(2):
        g.launch(stream=s)
        s.synchronize()
        scratch = torch.ones(1 << 20, device="cuda") * 3.0
        torch.cuda.synchronize()
        assert np.array_equal(x.cpu().numpy(), eager[k]), k
        del scratch
    q = b.eval(_dev(flat))
    torch.cuda.synchronize()
    qn = q.cpu().numpy()
    # same cells through the single-plan kernels
    q2 = p2.eval(_dev(f2))
    q3 = p3.eval(_dev(f3))
    torch.cuda.synchronize()
    assert np.array_equal(qn[:len(f2) * 1024], q2.cpu().numpy().reshape(-1))
    assert np.array_equal(qn[len(f2) * 1024:], q3.cpu().numpy().reshape(-1))
    s2, s3 = c4_sample(len(f2), len(f3))
    errs, errs_def = [], []
    for plan, fc, qc, sel in ((p2, f2, qn[:len(f2) * 1024], s2), (p3, f3, qn[len(f2) * 1024:], s3)):
        cells = fc[sel].astype(np.float64)
        got = qc.reshape(len(fc), -1)[sel]
        full = oracle_q(plan, fc[sel]).reshape(len(sel), -1)
        w = np.float32(plan.weights).astype(np.float64)
        defn = oracle.collide_near_equilibrium(plan.dim, plan.n, plan.ntilde, plan.dirs, w,
                                               cells.reshape((len(sel),) + (plan.n,) * plan.dim))
        errs.append(per_cell_rel_linf(got, full, plan.npts))
        errs_def.append(per_cell_rel_linf(got, defn.reshape(len(sel), -1), plan.npts))
    print("config4 near-eq: %d 2D + %d 3D cells, max rel err vs Q(f,f) %.2e / %.2e, vs definition %.2e / %.2e"
          % (len(s2), len(s3), errs[0].max(), errs[1].max(), errs_def[0].max(), errs_def[1].max()))
    assert max(e.max() for e in errs) <= TOL
    assert max(e.max() for e in errs_def) <= TOL
    # mixed batch: plain and near-equilibrium plans of every family together
    pf2 = gpu_lib.Plan(2, 32, 8.0, num_dirs=16)
    p64 = gpu_lib.Plan(2, 64, 8.0, num_dirs=8, mode=near)
    rng = np.random.default_rng(5)
    cells = [(p2, f2[0]), (pf2, f2[1]), (p3, f3[0]), (p64, workloads.noisy_local_maxwellian(rng, 2, 64, 8.0)),
             (pf2, f2[2]), (p2, f2[3])]
    mflat, moffs = _layout(cells)
    mb = gpu_lib.BatchPlan([c[0] for c in cells], moffs)
    mq = mb.eval(_dev(mflat))
    torch.cuda.synchronize()
    mq = mq.cpu().numpy()
    for (plan, a), o in zip(cells, moffs):
        single = plan.eval(_dev(a.reshape(1, -1)))
        torch.cuda.synchronize()
        assert_same_cell(plan, mq[o:o + plan.npts], single.cpu().numpy())


def test_rk2_graph_step(gpu_lib):
    """The two-stage TVD Runge-Kutta step (the paper's integrator, Sec. 4) as a
    captured graph: two replays against the same recursion on the oracle,
    gaps between cells untouched, mass of every cell kept."""
    import torch
    dt = 0.01
    p2 = gpu_lib.Plan(2, 32, 8.0, num_dirs=16)
    p3 = gpu_lib.Plan(3, 24, 8.0, num_dirs=16)
    rng = np.random.default_rng(61)
    cells = [(p2, workloads.noisy_local_maxwellian(rng, 2, 32, 8.0)) for _ in range(9)]
    cells += [(p3, workloads.noisy_local_maxwellian(rng, 3, 24, 8.0)) for _ in range(2)]
    flat, offs = _layout(cells)
    b = gpu_lib.BatchPlan([c[0] for c in cells], offs)
    x = _dev(flat)
    s = torch.cuda.Stream()
    g = gpu_lib.StepGraph(b, x, dt, s, scheme="rk2")
    ref = [c[1].astype(np.float32).astype(np.float64).reshape(-1) for c in cells]
    for step in range(2):
        g.launch(stream=s)
        s.synchronize()
        got = x.cpu().numpy()
        for k, ((plan, _), o) in enumerate(zip(cells, offs)):
            f0 = ref[k]
            f1 = f0 + dt * oracle_q(plan, f0.astype(np.float32)).reshape(-1)
            f2 = f1 + dt * oracle_q(plan, f1.astype(np.float32)).reshape(-1)
            ref[k] = 0.5 * (f0 + f2)
            cell = got[o:o + plan.npts].astype(np.float64)
            assert rel_linf(cell, ref[k]) <= 2e-6, (step, k, rel_linf(cell, ref[k]))
            assert abs(cell.sum() - ref[k].sum()) <= 1e-5 * ref[k].sum()
            ref[k] = cell      # continue from the GPU state (the oracle sees its FP32 values)
    mask = np.ones(len(flat), bool)
    for (plan, _), o in zip(cells, offs):
        mask[o:o + plan.npts] = False
    assert np.all(got[mask] == -7.0)
    with pytest.raises(gpu_lib.QdvmError):
        gpu_lib.StepGraph(b, x, dt, s, scheme=5)
    with pytest.raises(ValueError):
        gpu_lib.StepGraph(b, x, dt, s, scheme="rk4")


def test_one_shot_eval_batched(gpu_lib):
    """qdvm_eval_batched (build, evaluate, synchronise, destroy in one call)
    gives the persistent batch's result bit for bit, for Q and for the Euler
    update, and its cells agree with the oracle."""
    import torch
    p32 = gpu_lib.Plan(2, 32, 8.0, num_dirs=16)
    p64 = gpu_lib.Plan(2, 64, 8.0, num_dirs=8)
    p24 = gpu_lib.Plan(3, 24, 8.0, num_dirs=16)
    cells = [(p32, workloads.random_positive(1500 + i, 2, 32)[0]) for i in range(13)]
    cells += [(p64, workloads.random_positive(1600 + i, 2, 64)[0]) for i in range(3)]
    cells += [(p24, workloads.random_positive(1700 + i, 3, 24)[0]) for i in range(2)]
    order = np.random.default_rng(18).permutation(len(cells))
    cells = [cells[k] for k in order]
    flat, offs = _layout(cells)
    plans = [c[0] for c in cells]
    b = gpu_lib.BatchPlan(plans, offs)
    fd = _dev(flat)
    want = b.eval(fd, out=torch.full_like(fd, -7.0))
    torch.cuda.synchronize()
    out = torch.full_like(fd, -7.0)
    gpu_lib.eval_batched(plans, offs, fd, out)
    got = out.cpu().numpy()
    assert np.array_equal(got, want.cpu().numpy())
    for k in (0, len(cells) // 2, len(cells) - 1):
        plan, a = cells[k]
        o = offs[k]
        assert rel_linf(got[o:o + plan.npts], oracle_q(plan, a)) <= TOL
    # Euler update in place through the one-shot call
    x = _dev(flat)
    gpu_lib.eval_batched(plans, offs, x, x, dt=0.01)
    ref = _dev(flat)
    b.eval(ref, out=ref, dt=0.01)
    torch.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy(), ref.cpu().numpy())
    # empty batch: nothing to do
    gpu_lib.eval_batched([], [], fd, out)
