"""Launch shapes and the autotuner: every shape of the tuning space gives the
operator and its adjoint to the parity tolerance (1e-5 of max|Q|, the oracle
on the same inputs), the tuner keeps a valid shape, and its cache file
($QDVM_TUNE_CACHE) is written and read back."""
import os

import numpy as np
import pytest

from paper_1201_3986_amd import workloads
from parity_util import oracle_q, oracle_vjp, per_cell_rel_linf, rel_linf

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("d,n,P,batch", [(3, 32, 8, 2), (3, 16, 16, 3), (3, 16, 16, 40), (2, 32, 16, 19)])
def test_every_shape_gives_the_operator(gpu_lib, d, n, P, batch):
    import torch
    f = workloads.random_positive(4000 + n + batch, d, n, batch)
    c = np.random.default_rng(4001).standard_normal(f.shape).astype(np.float32)
    plan = gpu_lib.Plan(d, n, 8.0, num_dirs=P)
    ref = oracle_q(plan, f)
    rf, rw = oracle_vjp(plan, f, c)
    threads = (0, 1) if (d == 3 and n in (16, 32)) else (0,)
    splits = (0, 1, 2, 4, 8) if d == 3 else (0, 1)
    fd, cd = _dev(f), _dev(c)
    for radix in (0, 1):
        for t in threads:
            for gd in (1, 2, 4):
                for sp in splits:
                    for op in (0, 1):
                        plan.set_config(op, radix=radix, threads=t, split=sp, grid_div=gd)
                        assert plan.get_config(op) == dict(radix=radix, threads=t, split=sp, grid_div=gd)
                    q = plan.eval(fd)
                    gf, gw = plan.vjp(fd, cd)
                    torch.cuda.synchronize()
                    eq = per_cell_rel_linf(q.cpu().numpy(), ref, n ** d).max()
                    ef = per_cell_rel_linf(gf.cpu().numpy(), rf, n ** d).max()
                    ew = rel_linf(gw.cpu().numpy(), rw)
                    assert max(eq, ef, ew) <= TOL, (radix, t, gd, sp, eq, ef, ew)
    with pytest.raises(gpu_lib.QdvmError):
        plan.set_config(0, grid_div=3)
    with pytest.raises(gpu_lib.QdvmError):
        plan.set_config(0, split=9)
    if not (d == 3 and n in (16, 32)):
        with pytest.raises(gpu_lib.QdvmError):
            plan.set_config(0, threads=1)


def test_autotune_and_cache(gpu_lib, tmp_path, monkeypatch):
    import torch
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("QDVM_TUNE_CACHE", str(path))
    f = workloads.random_positive(4100, 3, 32, 6)
    plan = gpu_lib.Plan(3, 32, 8.0, num_dirs=8)
    plan.autotune(6)
    lines = path.read_text().splitlines()
    assert len(lines) == 2 and all(l.startswith("qdvm4:") for l in lines)
    c0, c1 = plan.get_config(0), plan.get_config(1)
    for c in (c0, c1):
        assert c["radix"] in (0, 1) and c["threads"] in (0, 1) and c["grid_div"] in (1, 2) and 0 <= c["split"] <= 8
    # a second plan of the same shape takes the cached shapes without timing
    plan2 = gpu_lib.Plan(3, 32, 8.0, num_dirs=8)
    plan2.autotune(6)
    assert plan2.get_config(0) == c0 and plan2.get_config(1) == c1
    assert len(path.read_text().splitlines()) == 2
    # another batch class gets its own entries
    plan2.autotune(600)
    assert len(path.read_text().splitlines()) == 4
    q = plan.eval(_dev(f))
    torch.cuda.synchronize()
    assert per_cell_rel_linf(q.cpu().numpy(), oracle_q(plan, f), 32 ** 3).max() <= TOL
    # defaults restored
    gpu_lib.load().qdvm_set_config(plan.handle, 0, None)
    assert plan.get_config(0) == dict(radix=1, threads=0, split=0, grid_div=1)
