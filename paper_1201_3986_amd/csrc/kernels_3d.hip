// HIP kernels (gfx950) of the fast DVM collision operator: 3D cells, the
// multiplier preparation, the grad_w reduction and the launch dispatch.
//
// Mouhot, Pareschi, Rey, Sec. 3.2: under the decoupling (3.3), the kernel modes
// split over lattice directions (3.6), and each direction of the operator
// (3.7) is a pair of convolutions of f -- along the line e_p Z (multiplier
// alpha_p) and over the plane e_p^perp (multiplier alpha'_p) -- multiplied
// pointwise, minus f times the convolution with alpha_p alpha'_p (the loss).
// Both multipliers are real and even, so one complex inverse transform of
// (alpha_p + i alpha'_p) fhat yields the line sum g_p in its real part and the
// plane sum h_p in its imaginary part; the losses of all directions are one
// transform of Lambda fhat with Lambda = sum_p w_p alpha_p alpha'_p:
//
//     Q = sum_p w_p g_p h_p - f * IFFT(Lambda fhat).
//
// Execution model.  A lane owns whole pencils (1-D lines of the grid) in
// VGPRs and transforms them with the unrolled in-register FFT; passing from
// one axis to the next is a transpose through LDS, real and imaginary parts in
// turn so the staging buffer is only n^d floats.  The spectrum of f is kept in
// a per-slot global scratch (L2 resident) and re-read for each direction.
//   2D (n <= 64): one lane per pencil, a cell is n lanes of one wave, the
//                 transposes never leave the wave.
//   3D: one cell per workgroup of T threads, each lane owns Q = n^2/T
//       pencils; transposes are workgroup-wide.
// Unnormalised transforms are used throughout; the 1/n^d factors are folded
// into the prepared job weights (W_j / n^{2d}) and into Lambda (/ n^d).
#include "cells_3d.h"

#include <type_traits>

namespace qdvm {

// Gain-accumulator elements per lane kept in LDS by the plain evaluation (the
// LDS behind the Dirichlet tables, shared with the reduction slots that only
// the other cell routines use).  n = 32 with one pencil per lane: 6 x 1024
// floats fit beside the transpose cube and the largest table (Nt = 15).
template <int N, int T>
constexpr int lacc3d()
{
    return (N == 32 && T == 1024) ? 6 : 0;
}

template <int N, int T, int RV, bool SPLIT>
__global__ __launch_bounds__(T) void k_eval3d(DevPlan pl, int batch, const float* f, float* q, float dt,
                                              DevScratch s)
{
    constexpr int NN = N * N, NPTS = NN * N;
    extern __shared__ float smem[];
    float* xb = smem;
    float* dtab = smem + N * N * (N + 1);
    double* red = (double*)(dtab + dtab_floats(pl));
    const int tid = threadIdx.x;
    load_dtab(dtab, pl, tid, T);
    __syncthreads();
    const rsrc_t rlam = make_rsrc(s.lam, NPTS * 4);
    Cell3D cl;
    cl.fh = make_rsrc(s.spec + (size_t)blockIdx.x * NPTS, NPTS * 8);
    // near-equilibrium mode: spectrum of g, and for n = 32 (two transforms do not fit in the
    // registers of 1024 threads) a staging area for the transform of g of each job
    constexpr bool STAGE = N == 32;
    const rsrc_t rgh = make_rsrc(SPLIT ? s.spec2 + (size_t)blockIdx.x * NPTS : s.spec, NPTS * 8);
    const rsrc_t rtg = make_rsrc(SPLIT ? s.spec2 + (size_t)(gridDim.x + blockIdx.x) * NPTS : s.spec, NPTS * 8);
    for (int cell = blockIdx.x; cell < batch; cell += gridDim.x) {
        cl.f = make_rsrc(f + (size_t)cell * NPTS, NPTS * 4);
        cl.q = make_rsrc(q + (size_t)cell * NPTS, NPTS * 4);
        if constexpr (SPLIT)
            cell3d_eval_split<N, T, RV, STAGE>(pl, cl, rgh, rtg, rlam, s.jobw, dt, xb, red, dtab, tid);
        else
            cell3d_eval<N, T, RV, lacc3d<N, T>()>(pl, cl, rlam, s.jobw, dt, xb, dtab, tid, 0, 1, true,
                                                  dtab + dtab_floats(pl));
    }
}

template <int N, int T, int RV>
__global__ __launch_bounds__(T) void k_vjp3d(DevPlan pl, int batch, const float* __restrict__ f,
                                             const float* __restrict__ c, float* __restrict__ g,
                                             DevScratch s)
{
    constexpr int NN = N * N, NPTS = NN * N;
    extern __shared__ float smem[];
    float* xb = smem;
    float* dtab = smem + N * N * (N + 1);
    float* red = dtab + dtab_floats(pl);
    const int tid = threadIdx.x;
    load_dtab(dtab, pl, tid, T);
    __syncthreads();
    const size_t slot = (size_t)blockIdx.x * NPTS;
    const float inv_n = 1.f / (float)NPTS;
    const float inv_n2 = inv_n * inv_n;
    const rsrc_t rlam = make_rsrc(s.lam, NPTS * 4);
    const rsrc_t rr = make_rsrc(s.spec2 + slot, NPTS * 8);
    const rsrc_t rsh = make_rsrc(s.acc + slot, NPTS * 8);
    Cell3D cl;
    cl.fh = make_rsrc(s.spec + slot, NPTS * 8);
    for (int cell = blockIdx.x; cell < batch; cell += gridDim.x) {
        cl.f = make_rsrc(f + (size_t)cell * NPTS, NPTS * 4);
        cl.q = make_rsrc(g + (size_t)cell * NPTS, NPTS * 4);
        const rsrc_t rc = make_rsrc(c + (size_t)cell * NPTS, NPTS * 4);
        // grad_w partials: row blockIdx accumulates this workgroup's cells
        cell3d_vjp<N, T, RV>(pl, cl, rc, rr, rsh, make_rsrc(s.acc + slot, 0), rlam, s.jobw,
                             s.gw_part + (size_t)blockIdx.x * pl.njobs,
                             cell == (int)blockIdx.x, inv_n2, inv_n, xb, red, dtab, tid);
    }
}

// Bilinear Q(g, f): one cell per workgroup, persistent over cells; spec holds
// the transforms of f, spec2 those of g.
template <int N, int T, int RV>
__global__ __launch_bounds__(T) void k_eval3d_bil(DevPlan pl, int batch, const float* g, const float* f, float* q,
                                                  float dt, DevScratch s)
{
    constexpr int NN = N * N, NPTS = NN * N;
    extern __shared__ float smem[];
    float* xb = smem;
    float* dtab = smem + N * N * (N + 1);
    const int tid = threadIdx.x;
    load_dtab(dtab, pl, tid, T);
    __syncthreads();
    const rsrc_t rlam = make_rsrc(s.lam, NPTS * 4);
    const rsrc_t rgh = make_rsrc(s.spec2 + (size_t)blockIdx.x * NPTS, NPTS * 8);
    Cell3D cl;
    cl.fh = make_rsrc(s.spec + (size_t)blockIdx.x * NPTS, NPTS * 8);
    for (int cell = blockIdx.x; cell < batch; cell += gridDim.x) {
        cl.f = make_rsrc(f + (size_t)cell * NPTS, NPTS * 4);
        cl.q = make_rsrc(q + (size_t)cell * NPTS, NPTS * 4);
        const rsrc_t rg = make_rsrc(g + (size_t)cell * NPTS, NPTS * 4);
        cell3d_eval_bilinear<N, T, RV, lacc3d<N, T>()>(pl, cl, rg, rgh, rlam, s.jobw, dt, xb, dtab, tid,
                                                       dtab + dtab_floats(pl));
    }
}

// ------------------------------------------------------------------ direction-split launches
// When a batch has fewer cells than the GPU has workgroup slots, the direction
// loop of each cell is spread over G workgroups (workgroup b: cell b / G, jobs
// b % G, b % G + G, ...).  Each computes the forward transform(s) itself, the
// first of them also the loss, and writes its part of Q (or grad_f) to its
// own buffer; k_combine adds the G parts in a fixed order.
template <int N, int T, int RV>
__global__ __launch_bounds__(T) void k_eval3d_js(DevPlan pl, int batch, int G, const float* f, DevScratch s)
{
    constexpr int NN = N * N, NPTS = NN * N;
    extern __shared__ float smem[];
    float* xb = smem;
    float* dtab = smem + N * N * (N + 1);
    const int tid = threadIdx.x;
    load_dtab(dtab, pl, tid, T);
    __syncthreads();
    const int cell = blockIdx.x / G, g = blockIdx.x % G;
    Cell3D cl;
    cl.f = make_rsrc(f + (size_t)cell * NPTS, NPTS * 4);
    cl.q = make_rsrc(s.part + ((size_t)g * batch + cell) * NPTS, NPTS * 4);
    cl.fh = make_rsrc(s.spec + (size_t)blockIdx.x * NPTS, NPTS * 8);
    cell3d_eval<N, T, RV, lacc3d<N, T>()>(pl, cl, make_rsrc(s.lam, NPTS * 4), s.jobw, 0.f, xb, dtab, tid, g, G,
                                          g == 0, dtab + dtab_floats(pl));
}

template <int N, int T, int RV>
__global__ __launch_bounds__(T) void k_vjp3d_js(DevPlan pl, int batch, int G, const float* __restrict__ f,
                                                const float* __restrict__ c, DevScratch s)
{
    constexpr int NN = N * N, NPTS = NN * N;
    extern __shared__ float smem[];
    float* xb = smem;
    float* dtab = smem + N * N * (N + 1);
    float* red = dtab + dtab_floats(pl);
    const int tid = threadIdx.x;
    load_dtab(dtab, pl, tid, T);
    __syncthreads();
    const int cell = blockIdx.x / G, g = blockIdx.x % G;
    const size_t slot = (size_t)blockIdx.x * NPTS;
    const float inv_n = 1.f / (float)NPTS;
    Cell3D cl;
    cl.f = make_rsrc(f + (size_t)cell * NPTS, NPTS * 4);
    cl.q = make_rsrc(s.part + ((size_t)g * batch + cell) * NPTS, NPTS * 4);
    cl.fh = make_rsrc(s.spec + slot, NPTS * 8);
    cell3d_vjp<N, T, RV>(pl, cl, make_rsrc(c + (size_t)cell * NPTS, NPTS * 4), make_rsrc(s.spec2 + slot, NPTS * 8),
                         make_rsrc(s.acc + slot, NPTS * 8), make_rsrc(s.acc + slot, 0), make_rsrc(s.lam, NPTS * 4),
                         s.jobw,
                         s.gw_part + (size_t)cell * pl.njobs, true, inv_n * inv_n, inv_n, xb, red, dtab, tid, g,
                         G, g == 0);
}

// out = sum_g part[g] (g ascending), or f + dt * sum when dt != 0; out may equal f.
__global__ void k_combine(int64_t total, int G, const float* __restrict__ part, const float* f, float* out, float dt)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        float acc = 0.f;
        for (int g = 0; g < G; ++g) acc += part[(size_t)g * total + i];
        out[i] = dt == 0.f ? acc : __builtin_fmaf(dt, acc, f[i]);
    }
}

// ------------------------------------------------------------------ prep
// Lambda/n^d at every spectral index and the job weights W_j / n^{2d}, from the
// per-direction weights w (W_j = w_p + w_pp for a 2D perpendicular pair).
__global__ void k_prep(DevPlan pl, const float* __restrict__ w, float* __restrict__ lam,
                       float* __restrict__ jobw)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = pl.n, npts = pl.npts;
    const double inv = 1.0 / (double)npts;
    if (idx < pl.njobs) {
        const JobDesc J = pl.jobs[idx];
        const double W = (double)w[J.p] + (J.pp >= 0 ? (double)w[J.pp] : 0.0);
        jobw[idx] = (float)(W * inv * inv);
    }
    if (idx >= npts) return;
    int K[3];
    if (pl.dim == 2) {
        K[1] = idx / n;
        K[0] = idx % n;
        K[2] = 0;
    } else {
        K[2] = idx / (n * n);
        const int pi = idx % (n * n);
        K[0] = pi / n;
        K[1] = pi % n;
    }
    double acc = 0.0;
    for (int jb = 0; jb < pl.njobs; ++jb) {
        const JobDesc J = pl.jobs[jb];
        const double W = (double)w[J.p] + (J.pp >= 0 ? (double)w[J.pp] : 0.0);
        int sd = J.e[0] * K[0] + J.e[1] * K[1] + J.e[2] * K[2];
        sd %= n;
        if (sd < 0) sd += n;
        const double al = (double)pl.dirichlet[(pl.ntilde + 1 + J.M) * n + sd];
        double ap;
        if (pl.dim == 2) {
            int t = -J.e[1] * K[0] + J.e[0] * K[1];
            t %= n;
            if (t < 0) t += n;
            ap = pl.dirichlet[J.M * n + t];
        } else {
            ap = pl.aperp[(size_t)jb * npts + idx];
        }
        acc += W * al * ap;
    }
    lam[idx] = (float)(acc * inv);
}

// The bilinear operator's multipliers: Lambda / n^d summed over the directions
// one by one (a 2D pair (e, e_perp) contributes w_e A_M(e.K) D_M(e_perp.K) +
// w_perp A_M(e_perp.K) D_M(e.K)) and the per-direction weights w_p / n^{2d}.
__global__ void k_prep_bil(DevPlan pl, const float* __restrict__ w, float* __restrict__ lam,
                           float* __restrict__ dirw)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = pl.n, npts = pl.npts;
    const double inv = 1.0 / (double)npts;
    if (idx < pl.P) dirw[idx] = (float)((double)w[idx] * inv * inv);
    if (idx >= npts) return;
    int K[3];
    if (pl.dim == 2) {
        K[1] = idx / n;
        K[0] = idx % n;
        K[2] = 0;
    } else {
        K[2] = idx / (n * n);
        const int pi = idx % (n * n);
        K[0] = pi / n;
        K[1] = pi % n;
    }
    double acc = 0.0;
    for (int jb = 0; jb < pl.njobs; ++jb) {
        const JobDesc J = pl.jobs[jb];
        int sd = J.e[0] * K[0] + J.e[1] * K[1] + J.e[2] * K[2];
        sd %= n;
        if (sd < 0) sd += n;
        const int arow = (pl.ntilde + 1 + J.M) * n;   // line multipliers A_M
        if (pl.dim == 2) {
            int t = -J.e[1] * K[0] + J.e[0] * K[1];
            t %= n;
            if (t < 0) t += n;
            // line e, plane e_perp; a paired perpendicular takes the two roles exchanged
            acc += (double)w[J.p] * (double)pl.dirichlet[arow + sd] * (double)pl.dirichlet[J.M * n + t];
            if (J.pp >= 0)
                acc += (double)w[J.pp] * (double)pl.dirichlet[arow + t] * (double)pl.dirichlet[J.M * n + sd];
        } else {
            acc += (double)w[J.p] * (double)pl.dirichlet[arow + sd] * pl.aperp[(size_t)jb * npts + idx];
        }
    }
    lam[idx] = (float)(acc * inv);
}

// grad_w[p] = sum over the partial rows of the job holding p (0 if none), in
// FP64: one workgroup per direction, thread t summing rows t, t + 256, ...,
// then a fixed tree over the threads (the order does not depend on timing).
__global__ __launch_bounds__(256) void k_gw_reduce(DevPlan pl, int rows, const int32_t* __restrict__ dir_job,
                                                   const double* __restrict__ part, float* __restrict__ gw)
{
    __shared__ double red[256];
    const int p = blockIdx.x, tid = threadIdx.x;
    const int jb = dir_job[p];
    double acc = 0.0;
    if (jb >= 0)
        for (int c = tid; c < rows; c += 256) acc += part[(size_t)c * pl.njobs + jb];
    red[tid] = acc;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if (tid < o) red[tid] += red[tid + o];
        __syncthreads();
    }
    if (tid == 0) gw[p] = (float)red[0];
}

// ------------------------------------------------------------------ dispatch
int device_cu_count()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

int num_variants(int, int) { return 2; }

// Radix order used when none is set: 3D n = 32 runs 4 x 8 pencils (fewer live
// registers in the one-pencil-per-lane job loop than 8 x 4), else variant 0.
int default_variant(int dim, int n) { return (dim == 3 && n == 32) ? 1 : 0; }

namespace {

template <int N>
constexpr int t3d()
{
    return N == 32 ? 1024 : (N == 24 ? 576 : (N == 16 ? 256 : 64));
}

// The alternative workgroup size of a 3D cell (two pencils per lane), a
// launch shape the autotuner may choose: n = 32 at 512 threads, n = 16 at 128;
// 0 where there is none.
template <int N>
constexpr int t3d_alt()
{
    return N == 32 ? 512 : (N == 16 ? 128 : 0);
}

// Calls f with std::integral_constant<int, T> for the chosen workgroup size.
template <int N, class F>
hipError_t with_threads(bool alt, F&& f)
{
    if constexpr (t3d_alt<N>() > 0) {
        if (alt) return f(std::integral_constant<int, t3d_alt<N>()>{});
    }
    return f(std::integral_constant<int, t3d<N>()>{});
}

// transpose buffer | Dirichlet tables | reduction slots (5 doubles per wave) and n Maxwellian
// factors, or the gain-accumulator elements of the plain evaluation
template <int N, int T = t3d<N>()>
size_t lds3d(int ntilde)
{
    const size_t tail = std::max<size_t>(2 * (5 * ((T + 63) / 64) + N), (size_t)lacc3d<N, T>() * T);
    const size_t bytes = sizeof(float) * ((size_t)N * N * (N + 1) + (size_t)2 * (ntilde + 1) * N + tail);
    // nine-wave workgroups (n = 24) run one per CU: a second resident one
    // measured slower (the barriers of the two interleave on the SIMDs)
    return T == 576 ? std::max<size_t>(bytes, 81 * 1024) : bytes;
}

// Spread each cell's direction loop over G workgroups.  Automatic (split 0):
// when the batch leaves more than half of the workgroup slots (cap) idle, G as
// large as the slots allow (at most 8 and the number of jobs).  split 1: never;
// split G >= 2: G workgroups per cell whenever batch * G fits in the slots.
void choose_split(const DevPlan& pl, int batch, int cap, LaunchInfo& li, int split)
{
    if (batch < 1 || pl.njobs < 2 || split == 1) return;
    int G;
    if (split >= 2) {
        G = std::min(split, pl.njobs);
        if ((int64_t)batch * G > cap) return;
    } else {
        if (2 * batch > cap) return;
        G = std::min(std::min(pl.njobs, 8), cap / batch);
    }
    if (G < 2) return;
    li.jsplit = G;
    li.grid = batch * G;
    li.slots = li.grid;
}

}  // namespace

#define QDVM_SWITCH_3D(N_, ...)                          \
    switch (N_) {                                          \
        case 8: { constexpr int N = 8; __VA_ARGS__; } break;      \
        case 16: { constexpr int N = 16; __VA_ARGS__; } break;    \
        case 24: { constexpr int N = 24; __VA_ARGS__; } break;    \
        case 32: { constexpr int N = 32; __VA_ARGS__; } break;    \
        default: return hipErrorInvalidValue;              \
    }

bool has_alt_threads(int dim, int n) { return dim == 3 && (n == 16 || n == 32); }

hipError_t launch_prep(const DevPlan& pl, const float* w, DevScratch s, hipStream_t st)
{
    const int threads = 256;
    const int n = std::max(pl.npts, pl.njobs);
    hipLaunchKernelGGL(k_prep, dim3((n + threads - 1) / threads), dim3(threads), 0, st, pl, w, s.lam, s.jobw);
    return hipGetLastError();
}

LaunchInfo eval_launch_info(const DevPlan& pl, int batch, int variant, LaunchLimits lim)
{
    LaunchInfo li;
    hipError_t e = hipSuccess;
    if (pl.dim == 2) {
        e = eval2d_info(pl, batch, variant, li, lim);
    } else {
        auto body = [&]() -> hipError_t {
            QDVM_SWITCH_3D(pl.n, {
                e = with_threads<N>(lim.threads != 0, [&](auto tc) -> hipError_t {
                    constexpr int T = decltype(tc)::value;
                    li.block = T;
                    li.lds = lds3d<N, T>(pl.ntilde);
                    hipError_t r;
                    if (pl.mode)
                        r = variant ? shaped_grid(k_eval3d<N, T, 1, true>, T, li.lds, batch, lim, li.grid)
                                    : shaped_grid(k_eval3d<N, T, 0, true>, T, li.lds, batch, lim, li.grid);
                    else
                        r = variant ? shaped_grid(k_eval3d<N, T, 1, false>, T, li.lds, batch, lim, li.grid)
                                    : shaped_grid(k_eval3d<N, T, 0, false>, T, li.lds, batch, lim, li.grid);
                    li.slots = li.grid;
                    if (r == hipSuccess && !pl.mode && lim.allow_split) {
                        int cap = 0;
                        r = variant ? occupancy_grid(k_eval3d_js<N, T, 1>, T, li.lds, 1 << 30, cap)
                                    : occupancy_grid(k_eval3d_js<N, T, 0>, T, li.lds, 1 << 30, cap);
                        choose_split(pl, batch, cap, li, lim.split);
                    }
                    return r;
                });
            });
            return e;
        };
        e = body();
    }
    if (e != hipSuccess) li.grid = 0;
    return li;
}

hipError_t launch_eval(const DevPlan& pl, int batch, const float* f, float* q, float dt, DevScratch s,
                       const LaunchInfo& li, int variant, hipStream_t st)
{
    if (pl.dim == 2) return launch_eval2d(pl, batch, f, q, dt, s, li, variant, st);
    QDVM_SWITCH_3D(pl.n, {
        return with_threads<N>(li.block != t3d<N>(), [&](auto tc) -> hipError_t {
            constexpr int T = decltype(tc)::value;
            const dim3 g(li.grid), b(T);
            if (li.jsplit > 1) {
                if (variant) hipLaunchKernelGGL((k_eval3d_js<N, T, 1>), g, b, li.lds, st, pl, batch, li.jsplit, f, s);
                else hipLaunchKernelGGL((k_eval3d_js<N, T, 0>), g, b, li.lds, st, pl, batch, li.jsplit, f, s);
                const int64_t total = (int64_t)batch * pl.npts;
                hipLaunchKernelGGL(k_combine, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 8192)), dim3(256),
                                   0, st, total, li.jsplit, s.part, f, q, dt);
            } else if (pl.mode) {
                if (variant) hipLaunchKernelGGL((k_eval3d<N, T, 1, true>), g, b, li.lds, st, pl, batch, f, q, dt, s);
                else hipLaunchKernelGGL((k_eval3d<N, T, 0, true>), g, b, li.lds, st, pl, batch, f, q, dt, s);
            } else {
                if (variant) hipLaunchKernelGGL((k_eval3d<N, T, 1, false>), g, b, li.lds, st, pl, batch, f, q, dt, s);
                else hipLaunchKernelGGL((k_eval3d<N, T, 0, false>), g, b, li.lds, st, pl, batch, f, q, dt, s);
            }
            return hipGetLastError();
        });
    });
    return hipErrorInvalidValue;
}

hipError_t launch_prep_bilinear(const DevPlan& pl, const float* w, DevScratch s, hipStream_t st)
{
    const int threads = 256;
    const int n = std::max(pl.npts, pl.P);
    hipLaunchKernelGGL(k_prep_bil, dim3((n + threads - 1) / threads), dim3(threads), 0, st, pl, w, s.lam, s.jobw);
    return hipGetLastError();
}

LaunchInfo bilinear_launch_info(const DevPlan& pl, int batch, int variant, LaunchLimits lim)
{
    LaunchInfo li;
    hipError_t e = hipSuccess;
    if (pl.dim == 2) {
        e = bil2d_info(pl, batch, variant, li, lim);
    } else {
        auto body = [&]() -> hipError_t {
            QDVM_SWITCH_3D(pl.n, {
                e = with_threads<N>(lim.threads != 0, [&](auto tc) -> hipError_t {
                    constexpr int T = decltype(tc)::value;
                    li.block = T;
                    li.lds = lds3d<N, T>(pl.ntilde);
                    hipError_t r = variant ? shaped_grid(k_eval3d_bil<N, T, 1>, T, li.lds, batch, lim, li.grid)
                                           : shaped_grid(k_eval3d_bil<N, T, 0>, T, li.lds, batch, lim, li.grid);
                    li.slots = li.grid;
                    return r;
                });
            });
            return e;
        };
        e = body();
    }
    if (e != hipSuccess) li.grid = 0;
    return li;
}

hipError_t launch_eval_bilinear(const DevPlan& pl, int batch, const float* g, const float* f, float* q, float dt,
                                DevScratch s, const LaunchInfo& li, int variant, hipStream_t st)
{
    if (pl.dim == 2) return launch_bil2d(pl, batch, g, f, q, dt, s, li, variant, st);
    QDVM_SWITCH_3D(pl.n, {
        return with_threads<N>(li.block != t3d<N>(), [&](auto tc) -> hipError_t {
            constexpr int T = decltype(tc)::value;
            if (variant)
                hipLaunchKernelGGL((k_eval3d_bil<N, T, 1>), dim3(li.grid), dim3(T), li.lds, st, pl, batch, g, f, q, dt,
                                   s);
            else
                hipLaunchKernelGGL((k_eval3d_bil<N, T, 0>), dim3(li.grid), dim3(T), li.lds, st, pl, batch, g, f, q, dt,
                                   s);
            return hipGetLastError();
        });
    });
    return hipErrorInvalidValue;
}

LaunchInfo vjp_launch_info(const DevPlan& pl, int batch, int variant, LaunchLimits lim)
{
    LaunchInfo li;
    hipError_t e = hipSuccess;
    if (pl.dim == 2) {
        e = vjp2d_info(pl, batch, variant, li, lim);
    } else {
        auto body = [&]() -> hipError_t {
            QDVM_SWITCH_3D(pl.n, {
                e = with_threads<N>(lim.threads != 0, [&](auto tc) -> hipError_t {
                    constexpr int T = decltype(tc)::value;
                    li.block = T;
                    li.lds = lds3d<N, T>(pl.ntilde);
                    hipError_t r = variant ? shaped_grid(k_vjp3d<N, T, 1>, T, li.lds, batch, lim, li.grid)
                                           : shaped_grid(k_vjp3d<N, T, 0>, T, li.lds, batch, lim, li.grid);
                    li.slots = li.grid;
                    if (r == hipSuccess && lim.allow_split) {
                        int cap = 0;
                        r = variant ? occupancy_grid(k_vjp3d_js<N, T, 1>, T, li.lds, 1 << 30, cap)
                                    : occupancy_grid(k_vjp3d_js<N, T, 0>, T, li.lds, 1 << 30, cap);
                        choose_split(pl, batch, cap, li, lim.split);
                    }
                    return r;
                });
            });
            return e;
        };
        e = body();
    }
    if (e != hipSuccess) li.grid = 0;
    return li;
}

int max_slots(const DevPlan& pl, int op, int variant, int threads)
{
    const int big = 1 << 28;
    LaunchLimits lim;
    lim.threads = threads;
    const LaunchInfo li = op == 0 ? eval_launch_info(pl, big, variant, lim)
                                  : (op == 1 ? vjp_launch_info(pl, big, variant, lim)
                                             : bilinear_launch_info(pl, big, variant, lim));
    if (li.grid <= 0) return 0;
    int slots = li.slots;
    if (op == 0 && pl.dim == 2 && !pl.mode) {
        // a 2D evaluation takes the per-job tables for large batches only: a
        // smaller batch may fill the (larger) grid of the shared-row kernel
        LaunchLimits rows = lim;
        rows.allow_jt = false;
        const LaunchInfo lr = eval_launch_info(pl, big, variant, rows);
        if (lr.grid <= 0) return 0;
        slots = std::max(slots, lr.slots);
    }
    if (pl.dim == 3 && op != 2 && !(op == 0 && pl.mode)) {
        // direction-split launches: one slot per workgroup, up to the split kernel's occupancy
        int cap = 0;
        hipError_t e = hipSuccess;
        auto body = [&]() -> hipError_t {
            QDVM_SWITCH_3D(pl.n, {
                e = with_threads<N>(threads != 0, [&](auto tc) -> hipError_t {
                    constexpr int T = decltype(tc)::value;
                    const size_t lds = lds3d<N, T>(pl.ntilde);
                    if (op == 0)
                        return variant ? occupancy_grid(k_eval3d_js<N, T, 1>, T, lds, 1 << 30, cap)
                                       : occupancy_grid(k_eval3d_js<N, T, 0>, T, lds, 1 << 30, cap);
                    return variant ? occupancy_grid(k_vjp3d_js<N, T, 1>, T, lds, 1 << 30, cap)
                                   : occupancy_grid(k_vjp3d_js<N, T, 0>, T, lds, 1 << 30, cap);
                });
            });
            return e;
        };
        if (body() != hipSuccess) return 0;
        slots = std::max(slots, cap);
    }
    return slots;
}

hipError_t launch_vjp(const DevPlan& pl, int batch, const float* f, const float* c, float* grad_f,
                      float* grad_w, const float* w, DevScratch s, const LaunchInfo& li, int variant,
                      hipStream_t st)
{
    (void)w;
    hipError_t e = hipSuccess;
    if (pl.dim == 2) {
        e = launch_vjp2d(pl, batch, f, c, grad_f, s, li, variant, st);
    } else {
        auto body = [&]() -> hipError_t {
            QDVM_SWITCH_3D(pl.n, {
                return with_threads<N>(li.block != t3d<N>(), [&](auto tc) -> hipError_t {
                    constexpr int T = decltype(tc)::value;
                    if (li.jsplit > 1) {
                        if (variant)
                            hipLaunchKernelGGL((k_vjp3d_js<N, T, 1>), dim3(li.grid), dim3(T), li.lds, st, pl, batch,
                                               li.jsplit, f, c, s);
                        else
                            hipLaunchKernelGGL((k_vjp3d_js<N, T, 0>), dim3(li.grid), dim3(T), li.lds, st, pl, batch,
                                               li.jsplit, f, c, s);
                        const int64_t total = (int64_t)batch * pl.npts;
                        hipLaunchKernelGGL(k_combine, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 8192)),
                                           dim3(256), 0, st, total, li.jsplit, s.part, (const float*)nullptr, grad_f,
                                           0.f);
                    } else if (variant)
                        hipLaunchKernelGGL((k_vjp3d<N, T, 1>), dim3(li.grid), dim3(T), li.lds, st, pl, batch, f, c,
                                           grad_f, s);
                    else
                        hipLaunchKernelGGL((k_vjp3d<N, T, 0>), dim3(li.grid), dim3(T), li.lds, st, pl, batch, f, c,
                                           grad_f, s);
                    return hipGetLastError();
                });
            });
            return hipErrorInvalidValue;
        };
        e = body();
    }
    if (e != hipSuccess) return e;
    if (grad_w) {
        // rows written: the slots that took a first cell (2D: row b * CPB + l
        // holds cell b * CPB + l first; 3D: row b holds cell b), or one per
        // cell in a direction-split launch (batch < slots there)
        const int rows = std::min(batch, li.slots);
        hipLaunchKernelGGL(k_gw_reduce, dim3(pl.P), dim3(256), 0, st, pl, rows, pl.dir_job, s.gw_part, grad_w);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace qdvm
