// Heterogeneous batch (gfx950): cells of different grid sizes and plans in
// persistent launches, with an optional forward-Euler epilogue q = f + dt Q.
//
// Spatially inhomogeneous kinetic codes apply the collision operator in every
// spatial cell, and the direction set may vary with position (Sec. 3.3, the
// adaptivity remark); the operator in each cell is the same as for a single
// cell.  The host sorts cells into work items -- one 3D cell, or up to
// blockDim/n consecutive 2D cells of one plan -- ordered by decreasing cost;
// each resident workgroup pops items from an atomic counter until the queue
// is empty, and runs the same per-cell device code as the uniform kernels.
// One launch covers every class of one block-size family:
//   256 threads: 2D n = 8, 16, 32
//   576 threads: 3D n = 24
//   512 threads: 2D n = 64 and 3D n = 32
#include "cells_2d.h"
#include "cells_3d.h"

namespace qdvm {

namespace {

// Values that are the same in every lane but were read from global memory (the
// compiler cannot prove that): readfirstlane moves them to scalar registers, so
// that buffer descriptors built from them need no per-lane loop.
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <class T>
__device__ __forceinline__ T* uni(T* p) { return (T*)(size_t)uni((int64_t)(size_t)p); }

__device__ __forceinline__ DevPlan uniform_plan(const DevPlan& p)
{
    DevPlan u;
    u.dim = uni(p.dim); u.n = uni(p.n); u.ntilde = uni(p.ntilde); u.P = uni(p.P); u.njobs = uni(p.njobs);
    u.npts = uni(p.npts); u.mode = uni(p.mode);
    u.jobs = uni(p.jobs); u.dirichlet = uni(p.dirichlet); u.aperp = uni(p.aperp); u.w_default = uni(p.w_default);
    u.dir_job = uni(p.dir_job); u.lam0 = uni(p.lam0); u.jobw0 = uni(p.jobw0);
    return u;
}

// LDS floats of the transpose buffers: eight 2D n=32 cells (256 threads), one
// 3D n=24 cell (576) or one 3D n=32 cell (512); every other class of a family
// fits inside.
__host__ __device__ constexpr int batched_xb_floats(int T)
{
    return T == 256 ? 8 * 32 * 33 : (T == 576 ? 24 * 24 * 25 : 32 * 32 * 33);
}
constexpr int kRedFloats = 2 * (5 * 9 + 32);   // 5 doubles per wave (up to 9 waves) and 32 Maxwellian factors

template <int N, int T, bool SPLIT>
__device__ __forceinline__ void batch_item_2d(const DevPlan& pl, const BatchItem& I, const BatchDev& b,
                                              const float* f, float* q, float dt, float* xbase,
                                              const float* dtab, float2* slot)
{
    constexpr int CPW = 64 / N, NPTS = N * N;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j = lane % N, local = wave * CPW + lane / N;
    const bool valid = local < I.count;
    const int64_t off = b.cell_off[I.first + (valid ? local : 0)];
    Item2D it;
    it.f = make_rsrc(f, b.fbytes);
    it.q = make_rsrc(q, b.fbytes);
    it.fh = make_rsrc(slot, (T / N) * NPTS * 8);
    it.vcell = (int)((off + j) * 4);
    it.vspec = (local * NPTS + j) * 8;
    const rsrc_t rlam = make_rsrc(pl.lam0, NPTS * 4);
    // at 512 threads the registers cannot hold two transforms of a 2D n = 64 job
    constexpr bool STAGE = T == 512;
    if (SPLIT && pl.mode)
        cell2d_eval_split<N, 0, STAGE>(pl, it, make_rsrc(slot + b.gslot, (T / N) * NPTS * 8),
                                       make_rsrc(slot + 2 * b.gslot, (T / N) * NPTS * 8), rlam, pl.jobw0, dt,
                                       valid, xbase + local * N * (N + 1), dtab, j);
    else
        cell2d_eval<N, 0>(pl, it, rlam, pl.jobw0, dt, valid, xbase + local * N * (N + 1), dtab, j,
                          make_rsrc(slot + b.fslot, (T / N) * NPTS * 8), b.fslot != 0 && pl.njobs > kFlushJobs);
}

template <int N, int T, bool SPLIT>
__device__ __forceinline__ void batch_item_3d(const DevPlan& pl, const BatchItem& I, const BatchDev& b,
                                              const float* f, float* q, float dt, float* xbase,
                                              const float* dtab, float2* slot, double* red)
{
    constexpr int NPTS = N * N * N;
    const int64_t off = uni(b.cell_off[I.first]);
    Cell3D cl;
    cl.f = make_rsrc(f + off, NPTS * 4);
    cl.q = make_rsrc(q + off, NPTS * 4);
    cl.fh = make_rsrc(slot, NPTS * 8);
    const rsrc_t rlam = make_rsrc(pl.lam0, NPTS * 4);
    constexpr bool STAGE = N == 32;
    if (SPLIT && pl.mode)
        cell3d_eval_split<N, T, 0, STAGE>(pl, cl, make_rsrc(slot + b.gslot, NPTS * 8),
                                          make_rsrc(slot + 2 * b.gslot, NPTS * 8), rlam, pl.jobw0, dt, xbase, red,
                                          dtab, threadIdx.x);
    else
        cell3d_eval<N, T, 0>(pl, cl, rlam, pl.jobw0, dt, xbase, dtab, threadIdx.x);
}

}  // namespace

// Drain the queue of one class.  Ticket k of a class is item k; the first
// round is static (workgroup g takes ticket g).  Later tickets come from the
// class's counter, which thread 0 bumps while the current item is being
// computed, so the atomic's latency is hidden -- or, when every item of the
// class costs the same, statically (g, g + grid, ...), which measured faster.  Each class runs its own loop,
// so that its registers are allocated for its own cell code only.
template <int C, int T, bool SPLIT>
__device__ __forceinline__ void drain_class(const BatchDev& b, const float* f, float* q, float dt, float* dtab,
                                            float* xbase, double* red, int* s_ticket, float2* slot, int& cur_plan)
{
    const int tid = threadIdx.x;
    __syncthreads();                          // the previous class's last ticket has been read
    int t = blockIdx.x;
    for (int k = 0;; ++k) {
        // t is uniform; readfirstlane makes that visible, so the item, its plan
        // and every buffer descriptor derived from them live in scalar registers
        t = __builtin_amdgcn_readfirstlane(t);
        if (t >= b.cls_count[C]) break;
        if (tid == 0)
            s_ticket[k & 1] = b.cls_static[C] ? t + (int)gridDim.x : (int)gridDim.x + atomicAdd(b.counter + C, 1);
        const BatchItem Iv = b.items[b.cls_first[C] + t];
        const BatchItem I = {uni(Iv.cls), uni(Iv.plan), uni(Iv.first), uni(Iv.count)};
        const DevPlan pl = uniform_plan(b.plans[I.plan]);
        if (I.plan != cur_plan) {
            __syncthreads();                  // the previous item no longer reads the table
            load_dtab(dtab, pl, tid, T);
            __syncthreads();
            cur_plan = I.plan;
        }
        if constexpr (C == BC_2D8) batch_item_2d<8, T, SPLIT>(pl, I, b, f, q, dt, xbase, dtab, slot);
        else if constexpr (C == BC_2D16) batch_item_2d<16, T, SPLIT>(pl, I, b, f, q, dt, xbase, dtab, slot);
        else if constexpr (C == BC_2D32) batch_item_2d<32, T, SPLIT>(pl, I, b, f, q, dt, xbase, dtab, slot);
        else if constexpr (C == BC_2D64) batch_item_2d<64, T, SPLIT>(pl, I, b, f, q, dt, xbase, dtab, slot);
        else if constexpr (C == BC_3D24) batch_item_3d<24, T, SPLIT>(pl, I, b, f, q, dt, xbase, dtab, slot, red);
        else batch_item_3d<32, T, SPLIT>(pl, I, b, f, q, dt, xbase, dtab, slot, red);
        // the next ticket is visible, and the item no longer uses LDS; the
        // other slot of s_ticket is written only after the next barrier
        __syncthreads();
        t = s_ticket[k & 1];
    }
}

// SPLIT: the batch holds near-equilibrium plans (a separate instantiation, so
// that the register allocation of plain batches is not affected).  The classes
// of a family are drained one after the other, the most expensive first; a
// workgroup that finds one queue empty moves on to the next.
template <int T, bool SPLIT>
__global__ __launch_bounds__(T) void k_batched(BatchDev b, const float* f, float* q, float dt)
{
    // dynamic LDS only, so that the Dirichlet rows start at LDS address 0 and
    // are aligned to 4n bytes: table | transpose buffers | reductions | tickets
    extern __shared__ float smem[];
    float* dtab = smem;
    float* xbase = smem + b.dtab_floats;
    double* red = (double*)(xbase + batched_xb_floats(T));   // block reductions of the near-equilibrium mode
    int* s_ticket = (int*)(xbase + batched_xb_floats(T) + kRedFloats);   // two slots
    float2* slot = b.spec + (size_t)blockIdx.x * b.slot_elems;
    int cur_plan = -1;
    if constexpr (T == 256) {
        if (b.cls_count[BC_2D32]) drain_class<BC_2D32, T, SPLIT>(b, f, q, dt, dtab, xbase, red, s_ticket, slot, cur_plan);
        if (b.cls_count[BC_2D16]) drain_class<BC_2D16, T, SPLIT>(b, f, q, dt, dtab, xbase, red, s_ticket, slot, cur_plan);
        if (b.cls_count[BC_2D8]) drain_class<BC_2D8, T, SPLIT>(b, f, q, dt, dtab, xbase, red, s_ticket, slot, cur_plan);
    } else if constexpr (T == 576) {
        drain_class<BC_3D24, T, SPLIT>(b, f, q, dt, dtab, xbase, red, s_ticket, slot, cur_plan);
    } else {
        if (b.cls_count[BC_3D32]) drain_class<BC_3D32, T, SPLIT>(b, f, q, dt, dtab, xbase, red, s_ticket, slot, cur_plan);
        if (b.cls_count[BC_2D64]) drain_class<BC_2D64, T, SPLIT>(b, f, q, dt, dtab, xbase, red, s_ticket, slot, cur_plan);
    }
}

// Second stage of the two-stage TVD Runge-Kutta step: f <- (f + f1) / 2 on the
// batch's cells only (gaps between cells stay untouched).  One workgroup per cell.
__global__ void k_average_cells(const int64_t* __restrict__ off, const int32_t* __restrict__ cnt, float* f,
                                const float* __restrict__ f1)
{
    const int64_t o = off[blockIdx.x];
    const int n = cnt[blockIdx.x];
    for (int i = threadIdx.x; i < n; i += blockDim.x) f[o + i] = 0.5f * (f[o + i] + f1[o + i]);
}

hipError_t launch_average_cells(const int64_t* off, const int32_t* cnt, int ncells, float* f, const float* f1,
                                hipStream_t st)
{
    if (ncells <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_average_cells, dim3(ncells), dim3(256), 0, st, off, cnt, f, f1);
    return hipGetLastError();
}

// The queue counter is cleared by a kernel (not a memset) so that the pair of
// launches can be captured in a graph and replayed.
__global__ void k_reset_counter(int32_t* counter)
{
    if (threadIdx.x < kNumClasses) counter[threadIdx.x] = 0;
}

namespace {

template <int T>
hipError_t family_info(int nitems, bool split, LaunchInfo& li, size_t dtab_floats)
{
    li.block = T;
    li.lds = sizeof(float) * (dtab_floats + batched_xb_floats(T) + kRedFloats + 4);
    // 576 threads: one workgroup per CU (a second resident nine-wave workgroup
    // measured slower: their barriers interleave on the SIMDs)
    if (T == 576) li.lds = std::max<size_t>(li.lds, 81 * 1024);
    hipError_t e = split ? occupancy_grid(k_batched<T, true>, T, li.lds, nitems, li.grid)
                         : occupancy_grid(k_batched<T, false>, T, li.lds, nitems, li.grid);
    li.slots = li.grid;
    return e;
}

template <int T>
void family_launch(const BatchDev& b, const LaunchInfo& li, const float* f, float* q, float dt, hipStream_t st)
{
    if (b.gslot != 0) hipLaunchKernelGGL((k_batched<T, true>), dim3(li.grid), dim3(T), li.lds, st, b, f, q, dt);
    else hipLaunchKernelGGL((k_batched<T, false>), dim3(li.grid), dim3(T), li.lds, st, b, f, q, dt);
}

}  // namespace

hipError_t batched_launch_info(int family, int nitems, bool split, LaunchInfo& li, size_t dtab_floats)
{
    switch (family) {
        case BF_256: return family_info<256>(nitems, split, li, dtab_floats);
        case BF_576: return family_info<576>(nitems, split, li, dtab_floats);
        case BF_512: return family_info<512>(nitems, split, li, dtab_floats);
        default: return hipErrorInvalidValue;
    }
}

size_t batched_slot_elems(int family)
{
    // spectra of one work item: eight 2D n=32 cells, one 3D n=24 cell, one 3D n=32 cell / eight 2D n=64 cells
    return family == BF_256 ? (size_t)8 * 32 * 32 : (family == BF_576 ? (size_t)24 * 24 * 24 : (size_t)32 * 32 * 32);
}

bool batch_uses_counter(const BatchDev& b)
{
    for (int c = 0; c < kNumClasses; ++c)
        if (b.cls_count[c] > 0 && !b.cls_static[c]) return true;
    return false;
}

hipError_t launch_batched(int family, const BatchDev& b, const LaunchInfo& li, const float* f, float* q, float dt,
                          hipStream_t st)
{
    // the queue counters are only read by classes whose tickets are dynamic
    if (batch_uses_counter(b)) {
        hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, b.counter);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    switch (family) {
        case BF_256: family_launch<256>(b, li, f, q, dt, st); break;
        case BF_576: family_launch<576>(b, li, f, q, dt, st); break;
        case BF_512: family_launch<512>(b, li, f, q, dt, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------- adaptive direction count
// Sec. 3.3 (remark after the complexity count): the number of directions may
// depend on the position, with fewer where the distribution is close to
// equilibrium.  The distance of a cell from equilibrium is the relative L1
// distance r = sum |f - M| / sum |f| to its Maxwellian M (the index-grid
// Maxwellian of its moments, FP64, as in the near-equilibrium mode; M = 0 when
// the cell has none, and r = 0 for a cell that is zero).

namespace {

__global__ void k_adapt_reset(int32_t* count)
{
    if (threadIdx.x < kMaxLevels) count[threadIdx.x] = 0;
}

// Level of a cell at distance r (the number of thresholds exceeded); also
// stores r and the level to the optional outputs.
__device__ __forceinline__ int adapt_level(const AdaptDev& a, int c, double r)
{
    int lv = 0;
    for (int l = 0; l + 1 < a.nlevels; ++l)
        if (r > (double)a.thr[l]) lv = l + 1;
    if (a.level) a.level[c] = lv;
    if (a.dist) a.dist[c] = (float)r;
    return lv;
}

// One cell's place in its level's queue (one atomic per cell).
__device__ __forceinline__ void adapt_enqueue(const AdaptDev& a, int c, double r)
{
    const int lv = adapt_level(a, c, r);
    const int pos = atomicAdd(a.count + lv, 1);
    a.queue[(int64_t)lv * a.ncells + pos] = a.cell_in[c];
}

// 3D cells: one workgroup per cell, two passes over the cell (moments, then
// the distance from the Maxwellian).
template <int D, int N>
__global__ __launch_bounds__(256) void k_adapt_classify(AdaptDev a, const float* __restrict__ f)
{
    constexpr int NP = D == 2 ? N * N : N * N * N;
    __shared__ double red[5 * 4];
    const int c = blockIdx.x, tid = threadIdx.x;
    const float* fc = f + a.cell_in[c];
    double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};   // mass, first moments (3), second moment
    for (int e = tid; e < NP; e += 256) {
        const int i0 = D == 2 ? e / N : e / (N * N), i1 = D == 2 ? e % N : (e / N) % N, i2 = D == 2 ? 0 : e % N;
        const double v = fc[e];
        s[0] += v;
        s[1] += i0 * v;
        s[2] += i1 * v;
        s[3] += i2 * v;
        s[4] += (double)(i0 * i0 + i1 * i1 + i2 * i2) * v;
    }
    block_sum5d<256>(s, red, tid);
    const double m0 = s[1] / s[0], m1 = s[2] / s[0], m2 = s[3] / s[0];
    const double var = (s[4] / s[0] - m0 * m0 - m1 * m1 - m2 * m2) / D;
    const bool ok = s[0] > 0.0 && var > 0.25 && __builtin_isfinite(var) && __builtin_isfinite(m0) &&
                    __builtin_isfinite(m1) && __builtin_isfinite(m2);
    const double norm = ok ? s[0] * pow(2.0 * kPi * var, -0.5 * D) : 0.0;
    const double inv2v = ok ? 0.5 / var : 0.0;
    // M = norm E0(i0) E1(i1) E2(i2), the one-dimensional factors in LDS
    __shared__ double ex[3][N];
    if (tid < N) {
        ex[0][tid] = exp(-(tid - m0) * (tid - m0) * inv2v);
        ex[1][tid] = exp(-(tid - m1) * (tid - m1) * inv2v);
        ex[2][tid] = D == 3 ? exp(-(tid - m2) * (tid - m2) * inv2v) : 1.0;
    }
    __syncthreads();
    double t[5] = {0.0, 0.0, 0.0, 0.0, 0.0};   // sum |f - M|, sum |f|
    for (int e = tid; e < NP; e += 256) {
        const int i0 = D == 2 ? e / N : e / (N * N), i1 = D == 2 ? e % N : (e / N) % N, i2 = D == 2 ? 0 : e % N;
        const double v = fc[e];
        const double M = ok ? norm * ex[0][i0] * ex[1][i1] * ex[2][i2] : 0.0;
        t[0] += fabs(v - M);
        t[1] += fabs(v);
    }
    block_sum5d<256>(t, red, tid);
    if (tid == 0) adapt_enqueue(a, c, t[1] > 0.0 ? t[0] / t[1] : 0.0);
}

// 2D cells: one wave per cell, the cell held in registers (n^2 / 64 values per
// lane, element e = lane + 64 k), wave-wide sums only.  A workgroup classifies
// 64 cells and claims their queue places with one atomic per level (per-cell
// atomics on a few counters serialise).  n <= 32: 16 waves per workgroup (four
// cells each), so that the grid of ncells / 64 workgroups fills four waves per
// SIMD; n = 64 (a cell takes 64 registers per lane): four waves.
template <int N>
constexpr int classify_threads() { return N <= 32 ? 1024 : 256; }

template <int N>
__global__ __launch_bounds__(classify_threads<N>()) void k_adapt_classify_2d(AdaptDev a, const float* __restrict__ f)
{
    constexpr int K = N * N / 64, CPB = 64, W = classify_threads<N>() / 64;
    __shared__ int s_lv[CPB];
    __shared__ int s_base[kMaxLevels];
    __shared__ double s_e0[W][N];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c0 = blockIdx.x * CPB;
    const int nc = a.ncells - c0 < CPB ? a.ncells - c0 : CPB;
    // the reads of a wave's next cell go out before the current one is
    // classified (each wave takes several cells in turn; their memory latency
    // would otherwise add up)
    // (n <= 32; at n = 64 the second copy of a cell does not fit in registers)
    constexpr bool PF = K <= 16;
    // the 64 cell offsets of the workgroup, one per lane (a cell's reads then
    // wait for no offset read of their own); an adaptive plan keeps f below
    // 2 GiB, so an element offset fits in 32 bits
    const int off = lane < nc ? (int)a.cell_in[c0 + lane] : 0;
    auto cell_ptr = [&](int jj) { return f + (uint32_t)__shfl(off, jj, 64); };
    float vn[K];
    if (PF && wave < nc) {
        const float* fc = cell_ptr(wave);
#pragma unroll
        for (int k = 0; k < K; ++k) vn[k] = fc[lane + 64 * k];
    }
    for (int j = wave; j < nc; j += W) {
        const int c = c0 + j;
        float v[K];
        if constexpr (PF) {
#pragma unroll
            for (int k = 0; k < K; ++k) v[k] = vn[k];
            if (j + W < nc) {
                const float* fc = cell_ptr(j + W);
#pragma unroll
                for (int k = 0; k < K; ++k) vn[k] = fc[lane + 64 * k];
            }
        } else {
            const float* fc = cell_ptr(j);
#pragma unroll
            for (int k = 0; k < K; ++k) v[k] = fc[lane + 64 * k];
        }
        // element e = lane + 64 k sits at i0 = h + (64 / n) k, i1 = lane mod n
        // (n divides 64): the moments follow from three per-lane sums over k
        constexpr int ST = 64 / N;
        const int h = lane / N, i1 = lane % N;
        double A = 0.0, B = 0.0, C = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double x = v[k];
            A += x;
            B = __builtin_fma((double)k, x, B);
            C = __builtin_fma((double)(k * k), x, C);
        }
        double s0 = A, s1 = __builtin_fma((double)ST, B, h * A), s2 = i1 * A;
        double sq = (double)(h * h + i1 * i1) * A + (double)(2 * h * ST) * B + (double)(ST * ST) * C;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            s0 += __shfl_xor(s0, o, 64);
            s1 += __shfl_xor(s1, o, 64);
            s2 += __shfl_xor(s2, o, 64);
            sq += __shfl_xor(sq, o, 64);
        }
        const double m0 = s1 / s0, m1 = s2 / s0;
        const double var = 0.5 * (sq / s0 - m0 * m0 - m1 * m1);
        const bool ok = s0 > 0.0 && var > 0.25 && __builtin_isfinite(var) && __builtin_isfinite(m0) &&
                        __builtin_isfinite(m1);
        const double norm = ok ? s0 / (2.0 * kPi * var) : 0.0;
        const double inv2v = ok ? 0.5 / var : 0.0;
        // M(i0, i1) = norm E0(i0) E1(i1): lane l computes E0(l mod n) and
        // E1(l mod n) (two exps per lane).  E1 is the lane's own; the n values
        // E0(i) go through a per-wave LDS row, read at immediate offsets.
        const double e0l = exp(-(i1 - m0) * (i1 - m0) * inv2v), e1 = exp(-(i1 - m1) * (i1 - m1) * inv2v);
        if (lane < N) s_e0[wave][lane] = e0l;
        wave_sync();
        const double* e0row = &s_e0[wave][h];
        double dsum = 0.0, fsum = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double x = v[k];
            const double M = ok ? norm * e0row[ST * k] * e1 : 0.0;
            dsum += fabs(x - M);
            fsum += fabs(x);
        }
        wave_sync();   // the row is rewritten for the wave's next cell
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            dsum += __shfl_xor(dsum, o, 64);
            fsum += __shfl_xor(fsum, o, 64);
        }
        if (lane == 0) s_lv[j] = adapt_level(a, c, fsum > 0.0 ? dsum / fsum : 0.0);
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t < a.nlevels) {
        int cnt = 0;
        for (int j = 0; j < nc; ++j) cnt += s_lv[j] == t;
        s_base[t] = cnt ? atomicAdd(a.count + t, cnt) : 0;
    }
    __syncthreads();
    if (t < nc) {
        const int lv = s_lv[t];
        int rank = 0;
        for (int j = 0; j < t; ++j) rank += s_lv[j] == lv;
        a.queue[(int64_t)lv * a.ncells + s_base[lv] + rank] = a.cell_in[c0 + t];
    }
}

// Persistent drain of the level queues of class C (one item: up to cpi cells
// of one level).  Items are numbered from the last level (the most
// directions) down and assigned statically; results do not depend on which
// cells share an item (each cell runs on its own lanes or workgroup).  SPLIT:
// some level plans are near-equilibrium plans (as for k_batched).
template <int C, int T, bool SPLIT>
__global__ __launch_bounds__(T) void k_adaptive(AdaptDev a, const float* f, float* q, float dt)
{
    extern __shared__ float smem[];
    float* dtab = smem;
    float* xbase = smem + a.b.dtab_floats;
    double* red = (double*)(xbase + batched_xb_floats(T));
    float2* slot = a.b.spec + (size_t)blockIdx.x * a.b.slot_elems;
    const int cpi = a.cpi, nl = uni(a.nlevels);
    int total = 0;
    for (int l = 0; l < nl; ++l) total += (uni(a.count[l]) + cpi - 1) / cpi;
    int cur_plan = -1;
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        int l = nl - 1, k = t, cnt = uni(a.count[l]);
        while (k >= (cnt + cpi - 1) / cpi) {
            k -= (cnt + cpi - 1) / cpi;
            --l;
            cnt = uni(a.count[l]);
        }
        const BatchItem I = {C, l, l * a.ncells + k * cpi, cnt - k * cpi < cpi ? cnt - k * cpi : cpi};
        const DevPlan pl = uniform_plan(a.b.plans[l]);
        if (l != cur_plan) {
            __syncthreads();                  // the previous item no longer reads the table
            load_dtab(dtab, pl, threadIdx.x, T);
            __syncthreads();
            cur_plan = l;
        }
        if constexpr (C == BC_2D8) batch_item_2d<8, T, SPLIT>(pl, I, a.b, f, q, dt, xbase, dtab, slot);
        else if constexpr (C == BC_2D16) batch_item_2d<16, T, SPLIT>(pl, I, a.b, f, q, dt, xbase, dtab, slot);
        else if constexpr (C == BC_2D32) batch_item_2d<32, T, SPLIT>(pl, I, a.b, f, q, dt, xbase, dtab, slot);
        else if constexpr (C == BC_2D64) batch_item_2d<64, T, SPLIT>(pl, I, a.b, f, q, dt, xbase, dtab, slot);
        else if constexpr (C == BC_3D24) batch_item_3d<24, T, SPLIT>(pl, I, a.b, f, q, dt, xbase, dtab, slot, red);
        else batch_item_3d<32, T, SPLIT>(pl, I, a.b, f, q, dt, xbase, dtab, slot, red);
        __syncthreads();                      // LDS free for the next item
    }
}

template <int C, int T>
hipError_t adaptive_info_t(int ncells, bool split, LaunchInfo& li, size_t dtab_floats)
{
    li.block = T;
    li.lds = sizeof(float) * (dtab_floats + batched_xb_floats(T) + kRedFloats + 4);
    if (T == 576) li.lds = std::max<size_t>(li.lds, 81 * 1024);   // one nine-wave workgroup per CU
    hipError_t e = split ? occupancy_grid(k_adaptive<C, T, true>, T, li.lds, ncells, li.grid)
                         : occupancy_grid(k_adaptive<C, T, false>, T, li.lds, ncells, li.grid);
    li.slots = li.grid;
    return e;
}

template <int C, int T>
void adaptive_drain(const AdaptDev& a, const LaunchInfo& li, const float* f, float* q, float dt, hipStream_t st)
{
    if (a.b.gslot != 0) hipLaunchKernelGGL((k_adaptive<C, T, true>), dim3(li.grid), dim3(T), li.lds, st, a, f, q, dt);
    else hipLaunchKernelGGL((k_adaptive<C, T, false>), dim3(li.grid), dim3(T), li.lds, st, a, f, q, dt);
}

}  // namespace

hipError_t adaptive_launch_info(int cls, int ncells, bool split, LaunchInfo& li, size_t dtab_floats)
{
    switch (cls) {
        case BC_2D8: return adaptive_info_t<BC_2D8, 256>(ncells, split, li, dtab_floats);
        case BC_2D16: return adaptive_info_t<BC_2D16, 256>(ncells, split, li, dtab_floats);
        case BC_2D32: return adaptive_info_t<BC_2D32, 256>(ncells, split, li, dtab_floats);
        case BC_2D64: return adaptive_info_t<BC_2D64, 512>(ncells, split, li, dtab_floats);
        case BC_3D24: return adaptive_info_t<BC_3D24, 576>(ncells, split, li, dtab_floats);
        case BC_3D32: return adaptive_info_t<BC_3D32, 512>(ncells, split, li, dtab_floats);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_adaptive(const AdaptDev& a, const LaunchInfo& li, const float* f, float* q, float dt,
                           hipStream_t st)
{
    hipLaunchKernelGGL(k_adapt_reset, dim3(1), dim3(64), 0, st, a.count);
    const unsigned w4 = (unsigned)((a.ncells + 63) / 64);   // 2D: 64 cells per workgroup
    switch (a.cls) {
        case BC_2D8: hipLaunchKernelGGL((k_adapt_classify_2d<8>), dim3(w4), dim3(classify_threads<8>()), 0, st, a, f); break;
        case BC_2D16: hipLaunchKernelGGL((k_adapt_classify_2d<16>), dim3(w4), dim3(classify_threads<16>()), 0, st, a, f); break;
        case BC_2D32: hipLaunchKernelGGL((k_adapt_classify_2d<32>), dim3(w4), dim3(classify_threads<32>()), 0, st, a, f); break;
        case BC_2D64: hipLaunchKernelGGL((k_adapt_classify_2d<64>), dim3(w4), dim3(classify_threads<64>()), 0, st, a, f); break;
        case BC_3D24: hipLaunchKernelGGL((k_adapt_classify<3, 24>), dim3(a.ncells), dim3(256), 0, st, a, f); break;
        case BC_3D32: hipLaunchKernelGGL((k_adapt_classify<3, 32>), dim3(a.ncells), dim3(256), 0, st, a, f); break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (a.cls) {
        case BC_2D8: adaptive_drain<BC_2D8, 256>(a, li, f, q, dt, st); break;
        case BC_2D16: adaptive_drain<BC_2D16, 256>(a, li, f, q, dt, st); break;
        case BC_2D32: adaptive_drain<BC_2D32, 256>(a, li, f, q, dt, st); break;
        case BC_2D64: adaptive_drain<BC_2D64, 512>(a, li, f, q, dt, st); break;
        case BC_3D24: adaptive_drain<BC_3D24, 576>(a, li, f, q, dt, st); break;
        case BC_3D32: adaptive_drain<BC_3D32, 512>(a, li, f, q, dt, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace qdvm
