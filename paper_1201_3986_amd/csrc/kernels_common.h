// Device helpers shared by the 2D and 3D collision kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fft_reg.h"
#include "qdvm_internal.h"

namespace qdvm {

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Keep the scheduler from hoisting a whole pencil of loads ahead of their use
// (which multiplies live registers): fence every 8 elements of a load loop.
#define QDVM_CHUNK_FENCE(k)                                            \
    do {                                                               \
        if (((k) & 7) == 7) __builtin_amdgcn_sched_barrier(0);         \
    } while (0)

// ------------------------------------------------------------ buffer access
// Per-element global accesses go through buffer instructions: the base and
// extent live in a wave-uniform descriptor (SGPRs), the lane's pencil offset
// in one VGPR and the element stride in the uniform soffset, so a pencil of n
// elements costs one address register instead of n.  Accesses outside
// [0, bytes) return 0 / are dropped by the hardware.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float bload(rsrc_t r, int voff, int soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ float2 bload2(rsrc_t r, int voff, int soff)
{
    // copy the elements to scalars first: bit-casting an ext-vector element
    // expression directly has been seen to read element 0 for both
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    const unsigned int lo = v[0], hi = v[1];
    return make_float2(__builtin_bit_cast(float, lo), __builtin_bit_cast(float, hi));
}
__device__ __forceinline__ void bstore(float x, rsrc_t r, int voff, int soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, x), r, voff, soff, 0);
}
__device__ __forceinline__ void bstore2(float2 x, rsrc_t r, int voff, int soff)
{
    const float fx = x.x, fy = x.y;
    u32x2 v;
    v[0] = __builtin_bit_cast(unsigned int, fx);
    v[1] = __builtin_bit_cast(unsigned int, fy);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, 0);
}

// Plan data lives in global memory; reading it through a global-address-space
// pointer keeps the compiler from using flat loads (which also count against
// the LDS wait counter) when the plan was itself read from memory.
template <class T>
__device__ __forceinline__ T gload(const T* p, int i)
{
    static_assert(sizeof(T) % 4 == 0, "word-sized plan records");
    const __attribute__((address_space(1))) int* w = (const __attribute__((address_space(1))) int*)(p + i);
    int words[sizeof(T) / 4];
#pragma unroll
    for (unsigned k = 0; k < sizeof(T) / 4; ++k) words[k] = w[k];
    T v;
    __builtin_memcpy(&v, words, sizeof(T));
    return v;
}

// Dirichlet table in LDS: the rows D_M(s) (M = 0..Nt, s = 0..n-1; alpha' in 2D)
// followed by the rows D_M(s) - 1 (alpha), so that neither multiplier costs an
// instruction per element.
__device__ __forceinline__ int dtab_floats(const DevPlan& pl) { return 2 * (pl.ntilde + 1) * pl.n; }
__device__ __forceinline__ void load_dtab(float* dtab, const DevPlan& pl, int tid, int nthreads)
{
    // D_M rows (plane multipliers in 2D), then the line multipliers A_M
    const int m = 2 * (pl.ntilde + 1) * pl.n;
    for (int i = tid; i < m; i += nthreads) dtab[i] = gload(pl.dirichlet, i);
}
__device__ __forceinline__ const float* dtab_alpha(const float* dtab, const DevPlan& pl)
{
    return dtab + (pl.ntilde + 1) * pl.n;
}

typedef __attribute__((address_space(3))) const float* lds_fptr;

// LDS byte address of a pointer into shared memory.
__device__ __forceinline__ uint32_t lds_byte_addr(const float* p) { return (uint32_t)(size_t)(lds_fptr)p; }

// Walk along one row of n floats in LDS, the index moving by a fixed step per
// element, modulo n.  When n is a power of two and the row starts at an LDS
// address that is a multiple of 4n bytes, the offset is carried in bytes
// without wrapping and the wrap plus the row address are one and-or per read.
template <int N>
struct RowWalk {
    static constexpr bool kPow2 = (N & (N - 1)) == 0;
    uint32_t row, off, step;
    __device__ __forceinline__ RowWalk(const float* rowp, int start, int stride)   // 0 <= start, stride < n
        : row(lds_byte_addr(rowp)), off(kPow2 ? 4u * start : (uint32_t)start),
          step(kPow2 ? 4u * stride : (uint32_t)stride) {}
    __device__ __forceinline__ float get() const
    {
        if constexpr (kPow2) {
            // row | (off & m) as one bitfield insert (row has no bits below 4n)
            uint32_t a;
            asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(a) : "s"(4u * N - 1), "v"(off), "v"(row));
            return *(lds_fptr)(size_t)a;
        }
        else return *(lds_fptr)(size_t)(row + 4u * off);
    }
    __device__ __forceinline__ void next()
    {
        off += step;
        if constexpr (!kPow2) off -= (off >= (uint32_t)N) ? (uint32_t)N : 0u;
    }
};

// Spectrum of a real field, stored as the half k <= n/2 of every pencil (a
// contiguous half of the slot, so the working set of the spectral scratch is
// halved): element k > n/2 of a pencil is the conjugate of element n - k of
// the mirrored pencil (-K in the other axes), fhat(-K) = conj fhat(K).
// STRIDE: byte distance between consecutive elements of a pencil.
template <int N, int STRIDE>
struct HalfSpec {
    rsrc_t r;
    int own, mir;   // byte offsets of the lane's pencil and of its mirror
    __device__ __forceinline__ float2 get(int k) const
    {
        if (k <= N / 2) return bload2(r, own, k * STRIDE);
        const float2 v = bload2(r, mir, (N - k) * STRIDE);
        return make_float2(v.x, -v.y);
    }
    __device__ __forceinline__ void put(const float2 (&z)[N]) const
    {
#pragma unroll
        for (int k = 0; k <= N / 2; ++k) bstore2(z[k], r, own, k * STRIDE);
    }
};

// Elements k0 .. k0 + C - 1 of the lane's pencil (byte stride S) of buffer r,
// all issued before any of them is used.  Left alone, the scheduler may wait
// for each read in turn: it cannot move a read past a store to a buffer it
// cannot tell apart from this one (a result written in place, a spectrum
// slot), nor always sees that the reads are independent.
template <int C>
__device__ __forceinline__ void load_run(float (&v)[C], rsrc_t r, int voff, int k0, int S)
{
#pragma unroll
    for (int i = 0; i < C; ++i) v[i] = bload(r, voff, (k0 + i) * S);
    __builtin_amdgcn_sched_barrier(0);
}

// A byte offset unchanged, but opaque to the optimiser: a later read of a cell
// through it is not merged with an earlier read of the same address, which
// would keep the whole pencil alive in registers in between.
__device__ __forceinline__ int reread(int v)
{
    asm volatile("" : "+v"(v));
    return v;
}

// The value unchanged, but opaque to the optimiser (no instruction is emitted):
// stops it from reusing an expensive expression across a long stretch of code
// where keeping the result alive would cost registers.
__device__ __forceinline__ double opaque(double v)
{
    asm volatile("" : "+v"(v));
    return v;
}

// grad_w partial of one job in a slot's FP64 row: the slot's first cell stores
// it, later cells add to it.  One thread owns the row and its cells come in a
// fixed order, so the sum is the same on every run; the add is an atomic
// read-modify-write performed at the device-coherent cache level, which cannot
// see a stale copy of the value this thread wrote before.
__device__ __forceinline__ void gw_accumulate(double* p, double v, bool first)
{
    if (first)
        *p = v;
    else
        atomicAdd(p, v);
}

template <int N>
__device__ __forceinline__ int modc(int x)
{
    x %= N;
    return x < 0 ? x + N : x;
}

// One pencil transform, fenced so that the scheduler does not interleave
// neighbouring pencils or phases (which multiplies the live temporaries).
template <int N, int RV, int SIGN>
__device__ __forceinline__ void fftp(float2 (&x)[N])
{
    __builtin_amdgcn_sched_barrier(0);
    Radix<N, RV>::template fft<SIGN>(x);
    __builtin_amdgcn_sched_barrier(0);
}


// Grid of a persistent launch: the occupancy-limited number of resident
// workgroups on the device, capped by the number of work items.
template <class K>
inline hipError_t occupancy_grid(K kernel, int block, size_t lds, int items, int& grid)
{
    hipError_t e = hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    int cus = device_cu_count();
    if (cus < 1) cus = 1;
    grid = std::min(items, per_cu * cus);
    if (grid < 1) grid = 1;
    return hipSuccess;
}

// Persistent grid of a kernel: the occupancy grid (capped by the items),
// divided by grid_div and capped by max_grid.
template <class K>
inline hipError_t shaped_grid(K kernel, int block, size_t lds, int items, const LaunchLimits& lim, int& grid)
{
    hipError_t e = occupancy_grid(kernel, block, lds, items, grid);
    if (e != hipSuccess) return e;
    if (lim.grid_div > 1) {
        int full = 0;
        e = occupancy_grid(kernel, block, lds, 1 << 30, full);
        if (e != hipSuccess) return e;
        grid = std::min(grid, std::max(1, full / lim.grid_div));
    }
    if (lim.max_grid > 0) grid = std::min(grid, lim.max_grid);
    return hipSuccess;
}

}  // namespace qdvm
