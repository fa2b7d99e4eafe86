"""GPU bilinear operator Q(g, f) (qdvm_eval_bilinear) against the FP64 oracle's
direct pair sum, element by element: relative L-infinity error <= 1e-5 of
max|Q(g, f)| per cell.  Grids of the paper's workloads (2D n = 64 with P = 16
and 32, 3D n = 32 with P = 8 and 16) and every other supported size, with
paired and unpaired 2D lines, ragged batches, per-call weights, the Euler
update of g in place, the diagonal Q(f, f) and mass conservation."""
import numpy as np
import pytest

import oracle
from paper_1201_3986_amd import workloads
from parity_util import assert_oracle_direction_set, per_cell_rel_linf, rel_linf

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def oracle_bil(plan, g32, f32, w=None):
    assert_oracle_direction_set(plan)
    weights = np.float32(plan.weights if w is None else w).astype(np.float64)
    return oracle.collide_bilinear(plan.dim, plan.n, plan.ntilde, plan.dirs, weights,
                                   np.asarray(g32, np.float32).astype(np.float64),
                                   np.asarray(f32, np.float32).astype(np.float64))


def _bil(plan, g, f, **kw):
    import torch
    out = plan.eval_bilinear(_dev(g), _dev(f), **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("P", [16, 32])
def test_2d_n64_workload(gpu_lib, P):
    # f and g from the two-Maxwellian family of the 2D n = 64 workload, drawn
    # independently; 37 cells: nine 4-cell items and a ragged tail
    f = workloads.two_maxwellians_batch(3101, 37, 64, noise=0.05)
    g = workloads.two_maxwellians_batch(3102, 37, 64, noise=0.05)
    plan = gpu_lib.Plan(2, 64, 8.0, num_dirs=P)
    q = _bil(plan, g, f).reshape(37, -1)
    errs = per_cell_rel_linf(q, oracle_bil(plan, g, f), 64 * 64)
    print("bilinear 2D n=64 P=%d: max cell rel err %.3e" % (P, errs.max()))
    assert errs.max() <= TOL


@pytest.mark.parametrize("P", [8, 16])
def test_3d_n32_workload(gpu_lib, P):
    f = workloads.three_gaussians_batch(3201, 3, 32)
    g = workloads.three_gaussians_batch(3202, 3, 32)
    plan = gpu_lib.Plan(3, 32, 8.0, num_dirs=P)
    q = _bil(plan, g, f).reshape(3, -1)
    errs = per_cell_rel_linf(q, oracle_bil(plan, g, f), 32 ** 3)
    print("bilinear 3D n=32 P=%d: max cell rel err %.3e" % (P, errs.max()))
    assert errs.max() <= TOL


# every supported size, with an odd number of 2D lines (an unpaired job), the
# Farey order 4 set of the 2D n = 16 workload and ragged batches
@pytest.mark.parametrize("d,n,kw,batch", [
    (2, 8, dict(num_dirs=4), 45), (2, 16, dict(farey_order=4), 19), (2, 32, dict(num_dirs=13), 11),
    (2, 64, dict(num_dirs=9), 5), (3, 8, dict(num_dirs=13), 4), (3, 16, dict(num_dirs=16), 3),
    (3, 24, dict(num_dirs=16), 2),
])
def test_sizes(gpu_lib, d, n, kw, batch):
    f = workloads.random_positive(3300 + n, d, n, batch)
    g = workloads.random_positive(3400 + n, d, n, batch)
    plan = gpu_lib.Plan(d, n, 8.0, **kw)
    q = _bil(plan, g, f)
    errs = per_cell_rel_linf(q, oracle_bil(plan, g, f), n ** d)
    print("bilinear d=%d n=%d %s batch=%d: max cell rel err %.3e" % (d, n, kw, batch, errs.max()))
    assert errs.max() <= TOL


@pytest.mark.parametrize("d,n,P", [(2, 32, 16), (3, 24, 16)])
def test_weights_euler_in_place_diagonal_mass(gpu_lib, d, n, P):
    import torch
    rng = np.random.default_rng(3500 + d)
    f = workloads.random_positive(3501 + d, d, n, 3)
    g = workloads.random_positive(3502 + d, d, n, 3)
    plan = gpu_lib.Plan(d, n, 8.0, num_dirs=P)
    # per-call weights (the plan is not modified)
    w = rng.uniform(0.2, 2.0, P).astype(np.float32) * np.float32(plan.weights)
    q = _bil(plan, g, f, w=_dev(w))
    assert per_cell_rel_linf(q, oracle_bil(plan, g, f, w=w), n ** d).max() <= TOL
    q0 = _bil(plan, g, f)
    ref0 = oracle_bil(plan, g, f).reshape(q0.shape)
    assert per_cell_rel_linf(q0, ref0, n ** d).max() <= TOL
    # Euler update of g, in place
    dt = 0.01
    x = _dev(g)
    plan.eval_bilinear(x, _dev(f), out=x, dt=dt)
    torch.cuda.synchronize()
    assert rel_linf(x.cpu().numpy(), g.astype(np.float64) + dt * ref0) <= 1e-6
    # out aliasing f
    y = _dev(f)
    plan.eval_bilinear(_dev(g), y, out=y)
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy(), q0)
    # diagonal: Q(f, f) through the bilinear kernel and through qdvm_eval
    qd = _bil(plan, f, f).reshape(3, -1)
    qe = plan.eval(_dev(f))
    torch.cuda.synchronize()
    ref_ff = oracle.collide(d, n, plan.ntilde, plan.dirs, np.float32(plan.weights).astype(np.float64),
                            f.astype(np.float64)).reshape(3, -1)
    assert per_cell_rel_linf(qd, ref_ff, n ** d).max() <= TOL
    assert per_cell_rel_linf(qe.cpu().numpy().reshape(3, -1), ref_ff, n ** d).max() <= TOL
    # mass: sum_i Q(g, f)_i = 0 for any g and f, relative to sum |Q|
    for c in range(3):
        cell = q0.reshape(3, -1)[c].astype(np.float64)
        assert abs(cell.sum()) <= 1e-6 * np.abs(ref0.reshape(3, -1)[c]).sum()


def test_errors_and_empty(gpu_lib):
    import torch
    plan = gpu_lib.Plan(2, 16, 8.0, num_dirs=8)
    a = torch.zeros(256 * 2, device="cuda")
    b = torch.zeros(256 * 3, device="cuda")
    with pytest.raises(ValueError):
        plan.eval_bilinear(a, b)
    e = torch.empty(0, device="cuda")
    assert plan.eval_bilinear(e, e).numel() == 0
    lib = gpu_lib.load()
    assert lib.qdvm_eval_bilinear(plan.handle, 1, None, None, None, None, 0.0, None) == gpu_lib.QDVM_EINVAL
