// HIP kernels (gfx950) of the fast DVM collision operator: 2D cells.
//
// Mouhot, Pareschi, Rey, Sec. 3.2: under the decoupling (3.3) the kernel modes
// split over lattice directions (3.6), and each direction of the operator
// (3.7) is a pair of convolutions of f -- along the line e_p Z (multiplier
// alpha_p) and along e_p^perp (multiplier alpha'_p) -- multiplied pointwise,
// minus f times the convolution with alpha_p alpha'_p (the loss).  Both
// multipliers are real and even, so one complex inverse transform of
// (alpha_p + i alpha'_p) fhat gives the line sum g_p as its real part and the
// perpendicular sum h_p as its imaginary part; the losses of all directions
// are one transform of Lambda fhat, Lambda = sum_p w_p alpha_p alpha'_p:
//
//     Q = sum_p w_p g_p h_p - f * IFFT(Lambda fhat).
//
// In 2D, alpha_p(K) = D_M(e.K) - 1 and alpha'_p(K) = D_M(e_perp.K) with the
// Dirichlet kernel D_M(s) = sum_{|m|<=M} cos(2 pi m s / n), so both come from
// one small LDS table.  A direction and its perpendicular share a transform
// (their unit-weight terms are equal, Remark 3.5), with weights added.
//
// Layout: a cell is n lanes of one wave, lane j owning one pencil in VGPRs.
//   real space: lane j holds column j,  z[i0] = f(i0, j)    (coalesced I/O)
//   spectrum:   lane j holds row K0 = j, z[K1] = fhat(j, K1); scratch and
//               tables are stored [K1][K0] so that lane loads are coalesced.
// Moving between axes is a transpose through LDS inside the wave.
// Transforms are unnormalised; 1/n^2 factors sit in Lambda and in the job
// weights W_j / n^4 prepared by k_prep.
#include "cells_2d.h"

namespace qdvm {

// 256 threads, 256/n cells per workgroup item, persistent over items.  SPLIT
// selects the near-equilibrium evaluation (second spectral buffer for g); JT
// (plain mode) gives every job its own weighted multiplier rows in LDS
// (build_job_table) in place of the shared Dirichlet table.
template <int N, int RV, bool SPLIT, bool JT = false>
__global__ __launch_bounds__(256) void k_eval2d(DevPlan pl, int batch, const float* f, float* q, float dt,
                                                DevScratch s)
{
    static_assert(!(SPLIT && JT), "job tables serve the plain mode");
    constexpr int CPW = 64 / N, CPB = 4 * CPW, SLOT = N * (N + 1), NPTS = N * N;
    extern __shared__ float smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j = lane % N, local = wave * CPW + lane / N;
    float* xb = smem + local * SLOT;
    float* dtab = smem + CPB * SLOT;
    if constexpr (JT) build_job_table<N>(dtab, pl, s.jobw, tid, blockDim.x);
    else load_dtab(dtab, pl, tid, blockDim.x);
    __syncthreads();
    const int nitems = (batch + CPB - 1) / CPB;
    const rsrc_t rlam = make_rsrc(s.lam, NPTS * 4);
    Item2D it;
    it.fh = make_rsrc(s.spec + (size_t)blockIdx.x * CPB * NPTS, CPB * NPTS * 8);
    it.vcell = (local * NPTS + j) * 4;
    it.vspec = (local * NPTS + j) * 8;
    // near-equilibrium mode: the spectrum of g per slot (spec2 also holds a staging set, which
    // these launches leave unused: at 256 threads both transforms of a job stay in registers);
    // plain mode with more than kFlushJobs jobs: the flushed gain sums (cell2d_eval)
    constexpr bool STAGE = false;
    const rsrc_t rgh = make_rsrc((SPLIT || pl.njobs > kFlushJobs) ? s.spec2 + (size_t)blockIdx.x * CPB * NPTS : s.spec,
                                 CPB * NPTS * 8);
    const rsrc_t rtg = make_rsrc(SPLIT ? s.spec2 + (size_t)(gridDim.x + blockIdx.x) * CPB * NPTS : s.spec,
                                 CPB * NPTS * 8);
    for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
        const int first = item * CPB;
        const int nvalid = min(CPB, batch - first);
        it.f = make_rsrc(f + (size_t)first * NPTS, nvalid * NPTS * 4);
        it.q = make_rsrc(q + (size_t)first * NPTS, nvalid * NPTS * 4);
        if constexpr (SPLIT && N != 64)   // n = 64: k_eval2d_pair
            cell2d_eval_split<N, RV, STAGE>(pl, it, rgh, rtg, rlam, s.jobw, dt, first + local < batch, xb, dtab, j);
        else if constexpr (!SPLIT)
            cell2d_eval<N, RV, JT>(pl, it, rlam, s.jobw, dt, first + local < batch, xb, dtab, j, rgh,
                                   pl.njobs > kFlushJobs, dtab);
    }
}

// Near-equilibrium mode at n = 64: one cell per workgroup of two waves
// (cell2d_eval_split_pair), persistent over cells.  The workgroup's barriers
// then pair only the two waves of one cell, and its LDS (two transpose slots
// and the Dirichlet tables, 40 KiB at the default truncation) lets four such
// workgroups share a CU.
template <int RV>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_eval2d_pair(
    DevPlan pl, int batch, const float* f, float* q, float dt, DevScratch s)
{
    constexpr int N = 64, SLOT = N * (N + 1), NPTS = N * N;
    extern __shared__ float smem[];
    const int tid = threadIdx.x, j = tid & 63;
    const bool fwave = __builtin_amdgcn_readfirstlane(tid >> 6) != 0;
    float* xg = smem;
    float* xf = smem + SLOT;
    float* dtab = smem + 2 * SLOT;
    load_dtab(dtab, pl, tid, blockDim.x);
    __syncthreads();
    const rsrc_t rlam = make_rsrc(s.lam, NPTS * 4);
    Item2D it;
    it.fh = make_rsrc(s.spec + (size_t)blockIdx.x * NPTS, NPTS * 8);
    it.vcell = j * 4;
    it.vspec = j * 8;
    const rsrc_t rgh = make_rsrc(s.spec2 + (size_t)blockIdx.x * NPTS, NPTS * 8);
    for (int cell = blockIdx.x; cell < batch; cell += gridDim.x) {
        it.f = make_rsrc(f + (size_t)cell * NPTS, NPTS * 4);
        it.q = make_rsrc(q + (size_t)cell * NPTS, NPTS * 4);
        cell2d_eval_split_pair<N, RV>(pl, it, rgh, rlam, s.jobw, dt, true, xg, xf, dtab, j, fwave);
    }
}

template <int N, int RV>
__global__ __launch_bounds__(256) void k_vjp2d(DevPlan pl, int batch, const float* __restrict__ f,
                                               const float* __restrict__ c, float* __restrict__ g,
                                               DevScratch s)
{
    constexpr int CPW = 64 / N, CPB = 4 * CPW, SLOT = N * (N + 1), NPTS = N * N;
    extern __shared__ float smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j = lane % N, local = wave * CPW + lane / N;
    float* xb = smem + local * SLOT;
    float* dtab = smem + CPB * SLOT;
    load_dtab(dtab, pl, tid, blockDim.x);
    __syncthreads();
    const int nitems = (batch + CPB - 1) / CPB;
    const float inv_n = 1.f / (float)NPTS;
    const float inv_n2 = inv_n * inv_n;
    const size_t sbase = (size_t)blockIdx.x * CPB * NPTS;
    const rsrc_t rlam = make_rsrc(s.lam, NPTS * 4);
    const rsrc_t rr = make_rsrc(s.spec2 + sbase, CPB * NPTS * 8);
    const rsrc_t rsh = make_rsrc(s.acc + sbase, CPB * NPTS * 8);
    const rsrc_t rnone = make_rsrc(s.acc + sbase, 0);
    Item2D it;
    it.fh = make_rsrc(s.spec + sbase, CPB * NPTS * 8);
    it.vcell = (local * NPTS + j) * 4;
    it.vspec = (local * NPTS + j) * 8;
    for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
        const int first = item * CPB;
        const int nvalid = min(CPB, batch - first);
        const int cell = first + local;
        const bool valid = cell < batch;
        it.f = make_rsrc(f + (size_t)first * NPTS, nvalid * NPTS * 4);
        it.q = make_rsrc(g + (size_t)first * NPTS, nvalid * NPTS * 4);
        const rsrc_t rc = make_rsrc(c + (size_t)first * NPTS, nvalid * NPTS * 4);
        // grad_w partials: row blockIdx * CPB + local accumulates this slot's cells
        cell2d_vjp<N, RV>(pl, it, rc, rr, rsh, rnone, rlam, s.jobw,
                          s.gw_part + ((size_t)blockIdx.x * CPB + local) * pl.njobs, item == (int)blockIdx.x,
                          valid, inv_n2, inv_n, xb, dtab, j);
    }
}

// Bilinear Q(g, f): 256 threads, 256/n cells per workgroup item, persistent
// over items; spec holds the transforms of f, spec2 those of g.  At least two
// waves per SIMD: left alone, one radix order at n = 64 takes two registers
// beyond the 256 of that occupancy.
template <int N, int RV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_eval2d_bil(DevPlan pl, int batch, const float* g, const float* f,
                                                    float* q, float dt, DevScratch s)
{
    constexpr int CPW = 64 / N, CPB = 4 * CPW, SLOT = N * (N + 1), NPTS = N * N;
    extern __shared__ float smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j = lane % N, local = wave * CPW + lane / N;
    float* xb = smem + local * SLOT;
    float* dtab = smem + CPB * SLOT;
    load_dtab(dtab, pl, tid, blockDim.x);
    __syncthreads();
    const int nitems = (batch + CPB - 1) / CPB;
    const rsrc_t rlam = make_rsrc(s.lam, NPTS * 4);
    Item2D it;
    it.fh = make_rsrc(s.spec + (size_t)blockIdx.x * CPB * NPTS, CPB * NPTS * 8);
    it.vcell = (local * NPTS + j) * 4;
    it.vspec = (local * NPTS + j) * 8;
    const rsrc_t rgh = make_rsrc(s.spec2 + (size_t)blockIdx.x * CPB * NPTS, CPB * NPTS * 8);
    for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
        const int first = item * CPB;
        const int nvalid = min(CPB, batch - first);
        it.f = make_rsrc(f + (size_t)first * NPTS, nvalid * NPTS * 4);
        it.q = make_rsrc(q + (size_t)first * NPTS, nvalid * NPTS * 4);
        const rsrc_t rg = make_rsrc(g + (size_t)first * NPTS, nvalid * NPTS * 4);
        cell2d_eval_bilinear<N, RV>(pl, it, rg, rgh, rlam, s.jobw, dt, first + local < batch, xb, dtab, j);
    }
}

// ------------------------------------------------------------------ dispatch
namespace {
template <int N>
size_t lds2d(int ntilde) { return sizeof(float) * ((size_t)(256 / N) * N * (N + 1) + (size_t)2 * (ntilde + 1) * N); }
template <int N>
size_t lds2d_jobs(int jt_floats) { return sizeof(float) * ((size_t)(256 / N) * N * (N + 1) + (size_t)jt_floats); }
}  // namespace

#define QDVM_SWITCH_2D(N_, ...)                          \
    switch (N_) {                                          \
        case 8: { constexpr int N = 8; __VA_ARGS__; } break;      \
        case 16: { constexpr int N = 16; __VA_ARGS__; } break;    \
        case 32: { constexpr int N = 32; __VA_ARGS__; } break;    \
        case 64: { constexpr int N = 64; __VA_ARGS__; } break;    \
        default: return hipErrorInvalidValue;              \
    }

hipError_t eval2d_info(const DevPlan& pl, int batch, int variant, LaunchInfo& li, const LaunchLimits& lim)
{
    hipError_t e = hipSuccess;
    QDVM_SWITCH_2D(pl.n, {
        li.block = 256;
        li.lds = lds2d<N>(pl.ntilde);
        const int items = (batch + 256 / N - 1) / (256 / N);
        if (pl.mode && N == 64) {
            li.block = 128;
            li.lds = sizeof(float) * ((size_t)2 * N * (N + 1) + (size_t)2 * (pl.ntilde + 1) * N);
            e = variant ? shaped_grid(k_eval2d_pair<1>, 128, li.lds, batch, lim, li.grid)
                        : shaped_grid(k_eval2d_pair<0>, 128, li.lds, batch, lim, li.grid);
            li.slots = li.grid;
            return e;
        }
        if (pl.mode)
            e = variant ? shaped_grid(k_eval2d<N, 1, true>, 256, li.lds, items, lim, li.grid)
                        : shaped_grid(k_eval2d<N, 0, true>, 256, li.lds, items, lim, li.grid);
        else {
            // n = 64 and 32: per-job tables when they fit in LDS and keep the
            // occupancy of the shared rows, or (n = 32) cost at most one wave of four
            // per SIMD and the batch fills at least two rounds of the persistent grid
            // (the tables cost registers at n = 32: measured slower at 4096 cells,
            // 0.047 against 0.042 ms, and faster at 32768, 0.278 against 0.297 ms; at
            // n = 64 a plan whose tables halve the occupancy, as with 16 or more jobs,
            // runs 1.5x slower with them)
            if constexpr (N == 64 || N == 32) {
                const size_t lds_jt = lds2d_jobs<N>(pl.jt_floats);
                if (lim.allow_jt && lds_jt <= kMaxLds) {
                    int full = 0, full_jt = 0;
                    e = variant ? occupancy_grid(k_eval2d<N, 1, false>, 256, li.lds, 1 << 30, full)
                                : occupancy_grid(k_eval2d<N, 0, false>, 256, li.lds, 1 << 30, full);
                    if (e != hipSuccess) return e;
                    li.jt = (variant ? occupancy_grid(k_eval2d<N, 1, false, true>, 256, lds_jt, 1 << 30, full_jt)
                                     : occupancy_grid(k_eval2d<N, 0, false, true>, 256, lds_jt, 1 << 30,
                                                      full_jt)) == hipSuccess &&
                            (full_jt >= full || (N == 32 && items >= 2 * full_jt && 4 * full_jt >= 3 * full));
                    if (li.jt) li.lds = lds_jt;
                }
            }
            if ((N == 64 || N == 32) && li.jt) {
                e = variant ? shaped_grid(k_eval2d<N, 1, false, true>, 256, li.lds, items, lim, li.grid)
                            : shaped_grid(k_eval2d<N, 0, false, true>, 256, li.lds, items, lim, li.grid);
            } else {
                e = variant ? shaped_grid(k_eval2d<N, 1, false>, 256, li.lds, items, lim, li.grid)
                            : shaped_grid(k_eval2d<N, 0, false>, 256, li.lds, items, lim, li.grid);
            }
        }
        li.slots = li.grid * (256 / N);
    });
    return e;
}

hipError_t launch_eval2d(const DevPlan& pl, int batch, const float* f, float* q, float dt, DevScratch s,
                         const LaunchInfo& li, int variant, hipStream_t st)
{
    QDVM_SWITCH_2D(pl.n, {
        const dim3 g(li.grid), b(256);
        if (pl.mode && N == 64) {
            if (variant) hipLaunchKernelGGL((k_eval2d_pair<1>), g, dim3(128), li.lds, st, pl, batch, f, q, dt, s);
            else hipLaunchKernelGGL((k_eval2d_pair<0>), g, dim3(128), li.lds, st, pl, batch, f, q, dt, s);
        } else if (pl.mode) {
            if (variant) hipLaunchKernelGGL((k_eval2d<N, 1, true>), g, b, li.lds, st, pl, batch, f, q, dt, s);
            else hipLaunchKernelGGL((k_eval2d<N, 0, true>), g, b, li.lds, st, pl, batch, f, q, dt, s);
        } else if ((N == 64 || N == 32) && li.jt) {
            if (variant) hipLaunchKernelGGL((k_eval2d<N, 1, false, true>), g, b, li.lds, st, pl, batch, f, q, dt, s);
            else hipLaunchKernelGGL((k_eval2d<N, 0, false, true>), g, b, li.lds, st, pl, batch, f, q, dt, s);
        } else {
            if (variant) hipLaunchKernelGGL((k_eval2d<N, 1, false>), g, b, li.lds, st, pl, batch, f, q, dt, s);
            else hipLaunchKernelGGL((k_eval2d<N, 0, false>), g, b, li.lds, st, pl, batch, f, q, dt, s);
        }
    });
    return hipGetLastError();
}

hipError_t bil2d_info(const DevPlan& pl, int batch, int variant, LaunchInfo& li, const LaunchLimits& lim)
{
    hipError_t e = hipSuccess;
    QDVM_SWITCH_2D(pl.n, {
        li.block = 256;
        li.lds = lds2d<N>(pl.ntilde);
        const int items = (batch + 256 / N - 1) / (256 / N);
        e = variant ? shaped_grid(k_eval2d_bil<N, 1>, 256, li.lds, items, lim, li.grid)
                    : shaped_grid(k_eval2d_bil<N, 0>, 256, li.lds, items, lim, li.grid);
        li.slots = li.grid * (256 / N);
    });
    return e;
}

hipError_t launch_bil2d(const DevPlan& pl, int batch, const float* g, const float* f, float* q, float dt,
                        DevScratch s, const LaunchInfo& li, int variant, hipStream_t st)
{
    QDVM_SWITCH_2D(pl.n, {
        if (variant)
            hipLaunchKernelGGL((k_eval2d_bil<N, 1>), dim3(li.grid), dim3(256), li.lds, st, pl, batch, g, f, q, dt, s);
        else
            hipLaunchKernelGGL((k_eval2d_bil<N, 0>), dim3(li.grid), dim3(256), li.lds, st, pl, batch, g, f, q, dt, s);
    });
    return hipGetLastError();
}

hipError_t vjp2d_info(const DevPlan& pl, int batch, int variant, LaunchInfo& li, const LaunchLimits& lim)
{
    hipError_t e = hipSuccess;
    QDVM_SWITCH_2D(pl.n, {
        li.block = 256;
        li.lds = lds2d<N>(pl.ntilde);
        const int items = (batch + 256 / N - 1) / (256 / N);
        e = variant ? shaped_grid(k_vjp2d<N, 1>, 256, li.lds, items, lim, li.grid)
                    : shaped_grid(k_vjp2d<N, 0>, 256, li.lds, items, lim, li.grid);
        li.slots = li.grid * (256 / N);
    });
    return e;
}

hipError_t launch_vjp2d(const DevPlan& pl, int batch, const float* f, const float* c, float* grad_f,
                        DevScratch s, const LaunchInfo& li, int variant, hipStream_t st)
{
    QDVM_SWITCH_2D(pl.n, {
        if (variant)
            hipLaunchKernelGGL((k_vjp2d<N, 1>), dim3(li.grid), dim3(256), li.lds, st, pl, batch, f, c, grad_f, s);
        else
            hipLaunchKernelGGL((k_vjp2d<N, 0>), dim3(li.grid), dim3(256), li.lds, st, pl, batch, f, c, grad_f, s);
    });
    return hipGetLastError();
}

}  // namespace qdvm
