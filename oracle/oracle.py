"""ctypes front end of the FP64 oracle (test infrastructure only).

The numerics live in ``qdvm_oracle.c`` (direct summation, no transforms).  This
module only compiles it with gcc, marshals numpy arrays and picks the
parameters the paper fixes:

* lines through 0 of the box [-order, order]^d, one primitive representative
  per line with its first nonzero component positive (Sec. 3.2, Farey series
  and the set A^{d-1}), listed by (|e|_inf, |e|_2^2, lexicographic);
* default weights a(k) = h^(2d-1) |k| / gcd(k), b = 1 (Sec. 3.2, after
  eq. (3.3)), which is h^(2d-1) |e_p|_2 on the line of e_p; or, with the delta
  line-weight profile, a(k) = h^(2d-2) / gcd(k) (w_p = h^(2d-2), the point
  k = m e_p weighted by 1/|m|);
* default truncation Nt = floor(n / (3 + sqrt 2)) (Sec. 4, the choice of Nt
  next to Table 1; the printed values 1, 3, 7, 14 for 8, 16, 32, 64 points).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qdvm_oracle.c")
_LIBDIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_LIBDIR, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP).  Returns the library path."""
    os.makedirs(_LIBDIR, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i32p = ctypes.POINTER(ctypes.c_int32)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_lines.argtypes = [ctypes.c_int, ctypes.c_int, i32p, ctypes.c_int]
        lib.oracle_lines.restype = ctypes.c_int
        lib.oracle_default_weights.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, i32p, ctypes.c_int, dp]
        ci = ctypes.c_int
        lib.oracle_collide.argtypes = [ci] * 4 + [i32p, dp, ci, ci, dp, dp]
        lib.oracle_collide_terms.argtypes = [ci] * 4 + [i32p, ci, dp, dp]
        lib.oracle_collide_bilinear.argtypes = [ci] * 4 + [i32p, dp, ci, ci, dp, dp, dp]
        lib.oracle_vjp.argtypes = [ci] * 4 + [i32p, dp, ci, ci, dp, dp, dp, dp]
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        _lib = lib
        return lib


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def lines(d: int, order: int) -> np.ndarray:
    """All lines of the box [-order, order]^d, canonical representatives, (count, d)."""
    lib = _load()
    cnt = lib.oracle_lines(d, order, None, 0)
    if cnt < 0:
        raise ValueError("bad dimension or order")
    out = np.zeros((cnt, d), dtype=np.int32)
    _, ptr = _i32(out)
    lib.oracle_lines(d, order, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), cnt)
    return out


def first_lines(d: int, count: int) -> np.ndarray:
    """The first `count` lines in canonical order."""
    order = 1
    while True:
        ls = lines(d, order)
        if len(ls) >= count:
            # every line of a larger order has a larger |e|_inf, so the prefix is stable
            return ls[:count].copy()
        order += 1


def default_weights(d: int, h: float, dirs, line_weight: int = 0) -> np.ndarray:
    lib = _load()
    dirs, dptr = _i32(dirs)
    w = np.zeros(len(dirs), dtype=np.float64)
    lib.oracle_default_weights(d, float(h), len(dirs), dptr, int(line_weight),
                               w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return w


def default_ntilde(n: int) -> int:
    return int(math.floor(n / (3.0 + math.sqrt(2.0))))


def _cells(f, d, n):
    f = np.asarray(f, dtype=np.float64)
    npts = n ** d
    if f.size % npts:
        raise ValueError("f size is not a multiple of n^d")
    return np.ascontiguousarray(f), f.size // npts


def collide(d, n, ntilde, dirs, w, f, line_weight=0) -> np.ndarray:
    """Q(f, f) by direct summation; f has shape (..., n, ..., n) or (batch*n^d,).
    line_weight 1: the term of k = m e_p carries w_p / |m| (delta quadrature)."""
    lib = _load()
    f, batch = _cells(f, d, n)
    dirs, dptr = _i32(dirs)
    w, wptr = _f64(w)
    q = np.zeros_like(f)
    lib.oracle_collide(d, n, ntilde, len(dirs), dptr, wptr, int(line_weight), batch,
                       f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                       q.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return q


def collide_bilinear(d, n, ntilde, dirs, w, g, f, line_weight=0) -> np.ndarray:
    """Q(g, f) by direct summation (gain g(i+k) f(i+l), loss g(i) f(i+k+l));
    g and f of the same shape, one or more cells."""
    lib = _load()
    g, batch = _cells(g, d, n)
    f, batch_f = _cells(f, d, n)
    if batch_f != batch:
        raise ValueError("g and f differ in size")
    dirs, dptr = _i32(dirs)
    w, wptr = _f64(w)
    q = np.zeros_like(f)
    P = ctypes.POINTER(ctypes.c_double)
    lib.oracle_collide_bilinear(d, n, ntilde, len(dirs), dptr, wptr, int(line_weight), batch, g.ctypes.data_as(P),
                                f.ctypes.data_as(P), q.ctypes.data_as(P))
    return q


def collide_terms(d, n, ntilde, dirs, f, line_weight=0) -> np.ndarray:
    """Unit-weight per-direction contributions Q_p for one cell, shape (P, n^d)."""
    lib = _load()
    f, batch = _cells(f, d, n)
    if batch != 1:
        raise ValueError("collide_terms takes one cell")
    dirs, dptr = _i32(dirs)
    out = np.zeros((len(dirs), n ** d), dtype=np.float64)
    lib.oracle_collide_terms(d, n, ntilde, len(dirs), dptr, int(line_weight),
                             f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def vjp(d, n, ntilde, dirs, w, f, c, line_weight=0):
    """(grad_f, grad_w) of <c, Q(f; w)>; grad_w summed over cells."""
    lib = _load()
    f, batch = _cells(f, d, n)
    c, batch_c = _cells(c, d, n)
    if batch_c != batch:
        raise ValueError("f and c differ in size")
    dirs, dptr = _i32(dirs)
    w, wptr = _f64(w)
    gf = np.zeros_like(f)
    gw = np.zeros(len(dirs), dtype=np.float64)
    P = ctypes.POINTER(ctypes.c_double)
    lib.oracle_vjp(d, n, ntilde, len(dirs), dptr, wptr, int(line_weight), batch, f.ctypes.data_as(P),
                   c.ctypes.data_as(P), gf.ctypes.data_as(P), gw.ctypes.data_as(P))
    return gf, gw


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(t: int) -> None:
    _load().oracle_set_num_threads(int(t))


def index_maxwellian(d: int, n: int, f) -> np.ndarray:
    """The Maxwellian of the near-equilibrium evaluation, per cell, in FP64.

    On the index grid i in {0..n-1}^d: mass s0 = sum f, mean mu = sum i f / s0,
    temperature var = (sum |i|^2 f / s0 - |mu|^2) / d, and
    M(i) = s0 (2 pi var)^(-d/2) exp(-|i - mu|^2 / (2 var)) (the Maxwellian of
    Sec. 2.1 written in grid units).  A cell with s0 <= 0, var <= 1/4 or
    non-finite moments gets M = 0.  Returns an array of the shape of f.
    """
    flat, batch = _cells(f, d, n)
    cells = flat.reshape(batch, n ** d)
    idx = np.stack(np.meshgrid(*([np.arange(n, dtype=np.float64)] * d), indexing="ij"), axis=-1).reshape(-1, d)
    r2 = np.sum(idx * idx, axis=1)
    out = np.zeros_like(cells)
    for c in range(cells.shape[0]):
        v = cells[c]
        s0 = v.sum()
        with np.errstate(all="ignore"):
            mu = (idx * v[:, None]).sum(axis=0) / s0
            var = ((r2 * v).sum() / s0 - np.dot(mu, mu)) / d
        if not (s0 > 0 and np.isfinite(var) and var > 0.25 and np.all(np.isfinite(mu))):
            continue
        dist2 = np.sum((idx - mu) ** 2, axis=1)
        out[c] = s0 * (2.0 * np.pi * var) ** (-d / 2.0) * np.exp(-dist2 / (2.0 * var))
    return out.reshape(np.shape(f))


def equilibrium_distance(d: int, n: int, f) -> np.ndarray:
    """Distance of each cell from equilibrium, FP64: r = sum |f - M| / sum |f|
    with M = index_maxwellian(f), and r = 0 for a cell that is zero.

    The measure by which the adaptive batch gives cells close to equilibrium
    fewer directions (the adaptivity remark of Sec. 3.3 names the criterion,
    closeness to equilibrium, but no formula; this relative L1 distance is the
    reading taken).  Returns one value per cell.
    """
    flat, batch = _cells(f, d, n)
    cells = flat.reshape(batch, n ** d)
    M = index_maxwellian(d, n, cells.reshape((batch,) + (n,) * d)).reshape(batch, n ** d)
    num = np.abs(cells - M).sum(axis=1)
    den = np.abs(cells).sum(axis=1)
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)


def adaptive_levels(r, thresholds) -> np.ndarray:
    """Level of each cell: how many of the increasing thresholds its distance
    exceeds (strictly).  The thresholds are compared as given (FP32 values
    promoted to FP64)."""
    t = np.asarray(thresholds, dtype=np.float32).astype(np.float64)
    r = np.asarray(r, dtype=np.float64)
    return np.array([int(np.sum(x > t)) for x in np.ravel(r)], dtype=np.int32)


def collide_near_equilibrium(d, n, ntilde, dirs, w, f, line_weight=0) -> np.ndarray:
    """Q(f, f) - Q(M, M) with M = index_maxwellian(f), both by direct summation."""
    M = index_maxwellian(d, n, f)
    return collide(d, n, ntilde, dirs, w, f, line_weight) - collide(d, n, ntilde, dirs, w, M, line_weight)
