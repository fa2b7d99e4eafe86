"""qdvm_eval_noalloc (the evaluation whose scratch is the library's static
device array, for callers that cannot allocate) against qdvm_eval, through the
C interface: two calls in a row on each plan, the second with a smaller batch,
each checked against qdvm_eval's result on the same cells (bit for bit in 2D,
where a cell's arithmetic does not depend on the launch shape; to the parity
tolerance, 1e-5 of max|Q|, in 3D, where qdvm_eval may split a small batch's
directions over several workgroups and add the parts in another FP32 order)
and sampled cells against the oracle (1e-5 of max|Q|)."""
import numpy as np
import pytest

from paper_1201_3986_amd import workloads
from parity_util import oracle_q, per_cell_rel_linf

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _both(plan, f, w=None, dt=0.0):
    import torch
    fd = _dev(f)
    wd = _dev(w) if w is not None else None
    ref = plan.eval(fd, w=wd, dt=dt)
    out = torch.full_like(fd, float("nan"))
    plan.eval_noalloc(fd, out, w=wd, dt=dt)
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(len(f), -1), ref.cpu().numpy().reshape(len(f), -1)


def test_scratch_size(gpu_lib):
    assert gpu_lib.load().qdvm_noalloc_scratch_bytes() == 32 << 20


@pytest.mark.parametrize("mode", ["full", "near_equilibrium"])
def test_noalloc_2d_n64_two_calls(gpu_lib, mode):
    # 4096 cells need 4096 spectral slots at the natural launch (more than the
    # static array holds): the call runs fewer persistent workgroups; then a
    # smaller batch with per-call weights
    plan = gpu_lib.Plan(2, 64, 8.0, num_dirs=16, mode=mode)
    base = workloads.two_maxwellians_batch(2202, 64, 64, noise=0.05)
    f1 = np.ascontiguousarray(np.tile(base, (64, 1, 1)))
    got, ref = _both(plan, f1)
    assert np.array_equal(got, ref)
    f2 = workloads.random_positive(2203, 2, 64, 37)
    w = np.random.default_rng(2204).uniform(0.5, 1.5, 16).astype(np.float32) * np.float32(plan.weights)
    got2, ref2 = _both(plan, f2, w=w)
    assert np.array_equal(got2, ref2)
    if mode == "full":
        assert per_cell_rel_linf(got2[[0, 36]], oracle_q(plan, f2[[0, 36]], w=w), 64 * 64).max() <= TOL
        assert per_cell_rel_linf(got[[0, 63]], oracle_q(plan, f1[[0, 63]]), 64 * 64).max() <= TOL


@pytest.mark.parametrize("mode", ["full", "near_equilibrium"])
def test_noalloc_3d_two_calls(gpu_lib, mode):
    import torch
    plan = gpu_lib.Plan(3, 32, 8.0, num_dirs=8, mode=mode)
    f1 = workloads.three_gaussians_batch(2301, 48, 32)
    got, ref = _both(plan, f1)
    assert per_cell_rel_linf(got, ref, 32 ** 3).max() <= TOL
    # smaller input, in place with the Euler update
    f2 = workloads.three_gaussians_batch(2302, 3, 32)
    x = _dev(f2)
    plan.eval_noalloc(x, x, dt=0.01)
    ref2 = plan.eval(_dev(f2), dt=0.01)
    torch.cuda.synchronize()
    assert per_cell_rel_linf(x.cpu().numpy().reshape(3, -1), ref2.cpu().numpy().reshape(3, -1), 32 ** 3).max() <= TOL
    if mode == "full":
        assert per_cell_rel_linf(got[[0, 47]], oracle_q(plan, f1[[0, 47]]), 32 ** 3).max() <= TOL
        ev = per_cell_rel_linf(x.cpu().numpy().reshape(3, -1)[[2]],
                               f2[[2]].reshape(1, -1).astype(np.float64) + 0.01 * oracle_q(plan, f2[[2]]).reshape(1, -1),
                               32 ** 3)
        assert ev.max() <= 1e-6


def test_noalloc_2d_n16_and_3d_n24(gpu_lib):
    p16 = gpu_lib.Plan(2, 16, 8.0, farey_order=4)
    f = workloads.random_positive(2401, 2, 16, 5000)
    got, ref = _both(p16, f)
    assert np.array_equal(got, ref)
    got, ref = _both(p16, f[:3])
    assert np.array_equal(got, ref)
    p24 = gpu_lib.Plan(3, 24, 8.0, num_dirs=16)
    f3 = workloads.random_positive(2402, 3, 24, 300)
    got, ref = _both(p24, f3)
    assert per_cell_rel_linf(got, ref, 24 ** 3).max() <= TOL
    got, ref = _both(p24, f3[:2])
    assert per_cell_rel_linf(got, ref, 24 ** 3).max() <= TOL
    assert per_cell_rel_linf(got[[1]], oracle_q(p24, f3[[1]]), 24 ** 3).max() <= TOL


def test_noalloc_errors(gpu_lib):
    lib = gpu_lib.load()
    plan = gpu_lib.Plan(2, 16, 8.0, num_dirs=8)
    st = lib.qdvm_eval_noalloc(None, 1, None, None, None, 0.0, None)
    assert st == gpu_lib.QDVM_EINVAL
    st = lib.qdvm_eval_noalloc(plan.handle, -1, None, None, None, 0.0, None)
    assert st == gpu_lib.QDVM_EINVAL
    st = lib.qdvm_eval_noalloc(plan.handle, 2, None, None, None, 0.0, None)
    assert st == gpu_lib.QDVM_EINVAL
    assert lib.qdvm_last_error()          # the error text names the problem
    assert lib.qdvm_eval_noalloc(plan.handle, 0, None, None, None, 0.0, None) == gpu_lib.QDVM_OK
