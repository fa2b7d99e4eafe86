"""The forward transform stage at 2D n = 16 (qdvm_transform_stage), both
methods -- the register FFT of the collision kernels and the DFT as FP32
matrix-core products -- against the definition of the DFT written out in
FP64 (fhat = W f W, W[a][b] = exp(-2 pi i a b / 16)), to 1e-6 of max|fhat|,
on a batch with a ragged tail of workgroups; also after inverse-forward round
trips in registers (the compute-bound form of the stage)."""
import numpy as np
import pytest

from paper_1201_3986_amd import workloads

pytestmark = pytest.mark.gpu


def dft_definition(f):
    n = f.shape[-1]
    a = np.arange(n)
    W = np.exp(-2j * np.pi * np.outer(a, a) / n)
    return np.einsum("ka,cab,lb->ckl", W, f.astype(np.float64), W)   # fhat[c][K0][K1]


@pytest.mark.parametrize("method,reps", [(0, 0), (1, 0), (0, 3), (1, 3)])
def test_stage_matches_the_dft(gpu_lib, method, reps):
    import torch
    f = workloads.two_maxwellians_batch(4200, 37, 16, noise=0.05)
    out = gpu_lib.transform_stage(torch.from_numpy(f).cuda(), method=method, reps=reps)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.complex128)             # [c][K1][K0]
    ref = np.transpose(dft_definition(f), (0, 2, 1))
    err = np.max(np.abs(got - ref), axis=(1, 2)) / np.max(np.abs(ref), axis=(1, 2))
    print("transform stage method %d reps %d: max cell rel err %.3e" % (method, reps, err.max()))
    assert err.max() <= 1e-6 * (1 + reps)


def test_stage_errors(gpu_lib):
    lib = gpu_lib.load()
    assert lib.qdvm_transform_stage(2, 2, 16, 1, 0, None, None, None) == gpu_lib.QDVM_EINVAL
    assert lib.qdvm_transform_stage(0, 2, 16, 1, 65, None, None, None) == gpu_lib.QDVM_EINVAL
    assert lib.qdvm_transform_stage(0, 2, 32, 1, 0, None, None, None) == gpu_lib.QDVM_EUNSUPPORTED
    assert lib.qdvm_transform_stage(1, 2, 16, 0, 0, None, None, None) == gpu_lib.QDVM_OK
