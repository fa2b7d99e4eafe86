// Heterogeneous batch (gfx950): cells of different grid sizes and plans in one
// persistent launch, with an optional forward-Euler epilogue q = f + dt Q.
//
// Spatially inhomogeneous kinetic codes apply the collision operator in every
// spatial cell, and the direction set may vary with position (Sec. 3.3, the
// adaptivity remark); the operator in each cell is the same as for a single
// cell.  The host sorts cells into work items -- one 3D cell, or up to
// blockDim/n consecutive 2D cells of one plan -- ordered by decreasing cost;
// each resident workgroup pops items from an atomic counter until the queue
// is empty, and runs the same per-cell device code as the uniform kernels.
// One launch covers every class of one block-size family:
//   576 threads: 2D n = 8, 16, 32 and 3D n = 24
//   512 threads: 2D n = 64 and 3D n = 32
#include "cells_2d.h"
#include "cells_3d.h"

namespace qdvm {

namespace {

// LDS floats of the transpose buffers: 18 2D n=32 cells (576 threads) or one 3D
// n=32 cell (512 threads); every other class of the family fits inside.
__host__ __device__ constexpr int batched_xb_floats(int T) { return T == 576 ? 18 * 32 * 33 : 32 * 32 * 33; }
constexpr int kRedFloats = 160;   // 16 waves x 5 doubles

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
    // registers of 576 / 512 threads hold the two transforms of a job up to n = 16
    constexpr bool STAGE = N >= 32;
    if (SPLIT && pl.mode)
        cell2d_eval_split<N, 0, STAGE>(pl, it, make_rsrc(slot + b.gslot, (T / N) * NPTS * 8),
                                       make_rsrc(slot + 2 * b.gslot, (T / N) * NPTS * 8), rlam, pl.jobw0, dt,
                                       valid, xbase + local * N * (N + 1), dtab, j);
    else
        cell2d_eval<N, 0>(pl, it, rlam, pl.jobw0, dt, valid, xbase + local * N * (N + 1), dtab, j);
}

template <int N, int T, bool SPLIT>
__device__ __forceinline__ void batch_item_3d(const DevPlan& pl, const BatchItem& I, const BatchDev& b,
                                              const float* f, float* q, float dt, float* xbase,
                                              const float* dtab, float2* slot, double* red)
{
    constexpr int NPTS = N * N * N;
    const int64_t off = b.cell_off[I.first];
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

// SPLIT: the batch holds near-equilibrium plans (a separate instantiation, so
// that the register allocation of plain batches is not affected).
template <int T, int MINB, bool SPLIT>
__global__ __launch_bounds__(T, MINB) void k_batched(BatchDev b, const float* f, float* q, float dt)
{
    extern __shared__ float smem[];
    __shared__ int s_item;
    float* dtab = smem;
    float* xbase = smem + b.dtab_floats;
    double* red = (double*)(xbase + batched_xb_floats(T));   // block reductions of the near-equilibrium mode
    float2* slot = b.spec + (size_t)blockIdx.x * b.slot_elems;
    const int tid = threadIdx.x;
    int cur_plan = -1;
    for (;;) {
        __syncthreads();                      // the previous item no longer reads LDS or s_item
        if (tid == 0) s_item = atomicAdd(b.counter, 1);
        __syncthreads();
        const int it = s_item;
        if (it >= b.nitems) break;            // uniform: every thread read the same ticket
        const BatchItem I = b.items[it];
        const DevPlan pl = b.plans[I.plan];
        if (I.plan != cur_plan) {
            for (int i = tid; i < (pl.ntilde + 1) * pl.n; i += T) dtab[i] = pl.dirichlet[i];
            __syncthreads();
            cur_plan = I.plan;
        }
        if constexpr (T == 576) {
            switch (I.cls) {
                case BC_2D8: batch_item_2d<8, T, SPLIT>(pl, I, b, f, q, dt, xbase, dtab, slot); break;
                case BC_2D16: batch_item_2d<16, T, SPLIT>(pl, I, b, f, q, dt, xbase, dtab, slot); break;
                case BC_2D32: batch_item_2d<32, T, SPLIT>(pl, I, b, f, q, dt, xbase, dtab, slot); break;
                case BC_3D24: batch_item_3d<24, T, SPLIT>(pl, I, b, f, q, dt, xbase, dtab, slot, red); break;
                default: break;
            }
        } else {
            switch (I.cls) {
                case BC_2D64: batch_item_2d<64, T, SPLIT>(pl, I, b, f, q, dt, xbase, dtab, slot); break;
                case BC_3D32: batch_item_3d<32, T, SPLIT>(pl, I, b, f, q, dt, xbase, dtab, slot, red); break;
                default: break;
            }
        }
    }
}

// The queue counter is cleared by a kernel (not a memset) so that the pair of
// launches can be captured in a graph and replayed.
__global__ void k_reset_counter(int32_t* counter) { *counter = 0; }

hipError_t batched_launch_info(int family, int nitems, bool split, LaunchInfo& li, size_t dtab_floats)
{
    hipError_t e;
    if (family == BF_576) {
        li.block = 576;
        li.lds = sizeof(float) * (dtab_floats + batched_xb_floats(576) + kRedFloats);
        e = split ? occupancy_grid(k_batched<576, 2, true>, 576, li.lds, nitems, li.grid)
                  : occupancy_grid(k_batched<576, 2, false>, 576, li.lds, nitems, li.grid);
    } else {
        li.block = 512;
        li.lds = sizeof(float) * (dtab_floats + batched_xb_floats(512) + kRedFloats);
        e = split ? occupancy_grid(k_batched<512, 1, true>, 512, li.lds, nitems, li.grid)
                  : occupancy_grid(k_batched<512, 1, false>, 512, li.lds, nitems, li.grid);
    }
    li.slots = li.grid;
    return e;
}

size_t batched_slot_elems(int family) { return family == BF_576 ? (size_t)18 * 32 * 32 : (size_t)32 * 32 * 32; }

hipError_t launch_batched(int family, const BatchDev& b, const LaunchInfo& li, const float* f, float* q, float dt,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, st, b.counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const bool split = b.gslot != 0;
    if (family == BF_576) {
        if (split) hipLaunchKernelGGL((k_batched<576, 2, true>), dim3(li.grid), dim3(576), li.lds, st, b, f, q, dt);
        else hipLaunchKernelGGL((k_batched<576, 2, false>), dim3(li.grid), dim3(576), li.lds, st, b, f, q, dt);
    } else {
        if (split) hipLaunchKernelGGL((k_batched<512, 1, true>), dim3(li.grid), dim3(512), li.lds, st, b, f, q, dt);
        else hipLaunchKernelGGL((k_batched<512, 1, false>), dim3(li.grid), dim3(512), li.lds, st, b, f, q, dt);
    }
    return hipGetLastError();
}

}  // namespace qdvm
