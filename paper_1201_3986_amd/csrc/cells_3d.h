// Device code of one 3D cell of the fast DVM collision operator (included by
// the uniform-batch and the heterogeneous-batch kernels).  The algebra is the
// one described at the top of kernels_2d.hip; in 3D the plane multiplier
// alpha'_p(K) = sum_{l.e_p = 0, |l|_inf <= Nt} cos(2 pi K.l / n) comes from a
// per-direction table built in FP64 on the host.
#pragma once
#include "kernels_common.h"

namespace qdvm {

// ------------------------------------------------------------------ 3D cell
// Pencil phases (element index e runs along the pencil):
//   X: pencil pi = y*n + z, e = x      (real space; coalesced I/O at x*n^2 + pi)
//   Y: pencil pi = x*n + z, e = y
//   Z: pencil pi = x*n + y, e = z      (spectral; scratch/tables at Kz*n^2 + pi)
// LDS address of (x, y, z): x*SX + y*(n+1) + z, SX = n*(n+1).
// n = 32 with one pencil per thread (1024 threads): in phases Y and Z a wave
// holds two x-slabs, and they are chosen as a slab and its mirror (x and -x;
// wave 0: the self-mirror slabs 0 and n/2), so that the spectral pencils
// (Kx, Ky) and (-Kx, -Ky) sit in one wave and the half-stored spectrum's mirror
// half can come by cross-lane shuffle.  Elsewhere slab s of phases Y and Z is
// x = s.
template <int N, int T>
constexpr bool mirror_slabs() { return N == 32 && T == N * N; }

template <int N, int T>
__device__ __forceinline__ int slab_x(int s)
{
    if constexpr (mirror_slabs<N, T>()) {
        const int w = s >> 1, h = s & 1;
        return h == 0 ? w : (w == 0 ? N / 2 : N - w);
    } else {
        return s;
    }
}

// Logical spectral pencil Kx n + Ky of the thread pencil pi (phase Z).
template <int N, int T>
__device__ __forceinline__ int spec_pi(int pi)
{
    return slab_x<N, T>(pi / N) * N + pi % N;
}

// Thread pencil that holds the mirror (-Kx, -Ky) of thread pencil pi.
template <int N, int T>
__device__ __forceinline__ int mirror_thread(int pi)
{
    if constexpr (mirror_slabs<N, T>()) {
        const int s = pi / N, w = s >> 1, h = s & 1;
        return (2 * w + (w == 0 ? h : 1 - h)) * N + (N - pi % N) % N;
    } else {
        const int kx = pi / N, ky = pi % N;
        return ((N - kx) % N) * N + (N - ky) % N;
    }
}

template <int N, int PH, int T = 0>
__device__ __forceinline__ int addr3(int pi, int e)
{
    constexpr int SY = N + 1, SX = N * (N + 1);
    const int a = PH == 0 ? pi / N : slab_x<N, T>(pi / N), b = pi % N;
    if (PH == 0) return e * SX + a * SY + b;
    if (PH == 1) return a * SX + e * SY + b;
    return a * SX + b * SY + e;
}

// Exchange between two phases through the padded LDS cube, real parts then
// imaginary parts.  LEAD: begin with a workgroup barrier (needed when another
// wave may still be reading the rows this one writes).
template <int N, int T, int Q, int PA, int PB, bool LEAD = true>
__device__ __forceinline__ void block_transpose(float2 (&z)[Q][N], float* xb, int tid)
{
#pragma unroll
    for (int part = 0; part < 2; ++part) {
        if (part || LEAD) __syncthreads();
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int e = 0; e < N; ++e) xb[addr3<N, PA, T>(tid + q * T, e)] = part ? z[q][e].y : z[q][e].x;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int e = 0; e < N; ++e) {
                const float v = xb[addr3<N, PB, T>(tid + q * T, e)];
                if (part) z[q][e].y = v;
                else z[q][e].x = v;
            }
    }
}

// Phases Y and Z give a lane the same x (pencil pi = x n + b in both).  When n
// divides 64 the n lanes of an x-slab sit in one wave, so the Y <-> Z exchange
// only touches the LDS rows x of the wave's own slabs and needs no workgroup
// barrier; phase X <-> Y changes the slab of a lane and stays block-wide.
template <int N>
constexpr bool local_yz() { return 64 % N == 0; }

template <int N, int T, int Q, int PA, int PB>
__device__ __forceinline__ void wave_transpose(float2 (&z)[Q][N], float* xb, int tid)
{
#pragma unroll
    for (int part = 0; part < 2; ++part) {
        if (part) wave_sync();
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int e = 0; e < N; ++e) xb[addr3<N, PA, T>(tid + q * T, e)] = part ? z[q][e].y : z[q][e].x;
        wave_sync();
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int e = 0; e < N; ++e) {
                const float v = xb[addr3<N, PB, T>(tid + q * T, e)];
                if (part) z[q][e].y = v;
                else z[q][e].x = v;
            }
    }
}

// Forward: X -> Y block-wide (it begins with a barrier: the previous phase may
// have read any row), Y -> Z inside the wave (after the X -> Y reads each wave
// only touches its own rows).
template <int N, int T, int Q, int RV>
__device__ __forceinline__ void fwd3d(float2 (&z)[Q][N], float* xb, int tid)
{
#pragma unroll
    for (int q = 0; q < Q; ++q) fftp<N, RV, -1>(z[q]);
    block_transpose<N, T, Q, 0, 1>(z, xb, tid);
#pragma unroll
    for (int q = 0; q < Q; ++q) fftp<N, RV, -1>(z[q]);
    if constexpr (local_yz<N>()) wave_transpose<N, T, Q, 1, 2>(z, xb, tid);
    else block_transpose<N, T, Q, 1, 2>(z, xb, tid);
#pragma unroll
    for (int q = 0; q < Q; ++q) fftp<N, RV, -1>(z[q]);
}

// Inverse: one barrier, then Z -> Y inside the wave and Y -> X block-wide
// (whose first writes go to the wave's own rows, so it needs no leading
// barrier of its own).
template <int N, int T, int Q, int RV>
__device__ __forceinline__ void inv3d(float2 (&z)[Q][N], float* xb, int tid)
{
#pragma unroll
    for (int q = 0; q < Q; ++q) fftp<N, RV, 1>(z[q]);
    if constexpr (local_yz<N>()) {
        __syncthreads();
        wave_transpose<N, T, Q, 2, 1>(z, xb, tid);
    } else {
        block_transpose<N, T, Q, 2, 1>(z, xb, tid);
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) fftp<N, RV, 1>(z[q]);
    block_transpose<N, T, Q, 1, 0, !local_yz<N>()>(z, xb, tid);
#pragma unroll
    for (int q = 0; q < Q; ++q) fftp<N, RV, 1>(z[q]);
}

// FP64 sum over the workgroup (uniform result), for the grad_w partials: one
// cell's partial adds 1024 lanes' terms that largely cancel, and an FP32 tree
// over them leaves ~1e-5 of the result (2e-5 measured for a single direction at
// n = 32, 3e-7 in FP64).  red: 8-byte aligned, one double per wave.  The wave
// sums use swizzles, not lane shuffles: an FP64 shuffle chain on this per-job
// path made the adjoint of 64 n = 32 cells 8 % slower.
// FP64 sum over the 64 lanes of a wave (uniform result): xor swizzles of the two
// 32-bit halves within each half-wave, then the two half-waves by readlane.
__device__ __forceinline__ double wave_sumd(double v)
{
#define QDVM_SWZ_ADDD(pat)                                                                        \
    do {                                                                                          \
        const unsigned long long b = __builtin_bit_cast(unsigned long long, v);                   \
        const unsigned lo = (unsigned)__builtin_amdgcn_ds_swizzle((int)(unsigned)b, pat);         \
        const unsigned hi = (unsigned)__builtin_amdgcn_ds_swizzle((int)(unsigned)(b >> 32), pat); \
        v += __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);                    \
    } while (0)
    QDVM_SWZ_ADDD(0x041F);   // and 0x1f, xor 1
    QDVM_SWZ_ADDD(0x081F);   // xor 2
    QDVM_SWZ_ADDD(0x101F);   // xor 4
    QDVM_SWZ_ADDD(0x201F);   // xor 8
    QDVM_SWZ_ADDD(0x401F);   // xor 16
#undef QDVM_SWZ_ADDD
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned a0 = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, 0);
    const unsigned a1 = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 0);
    const unsigned c0 = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, 32);
    const unsigned c1 = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 32);
    return __builtin_bit_cast(double, ((unsigned long long)a1 << 32) | a0) +
           __builtin_bit_cast(double, ((unsigned long long)c1 << 32) | c0);
}

template <int T>
__device__ __forceinline__ double block_sumd(double v, double* red, int tid)
{
    v = wave_sumd(v);
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < (T + 63) / 64; ++w) t += red[w];
    return t;
}

// Buffers of one 3D cell: lane pencil pi = tid + q*T, element e at pi + e*n^2.
struct Cell3D {
    rsrc_t f, q, fh;
};

// Half-stored spectrum of one 3D cell slot at pencil pi = Kx n + Ky (mirror
// pencil (-Kx, -Ky)).
template <int N>
__device__ __forceinline__ HalfSpec<N, N * N * 8> half3d(rsrc_t r, int pi)
{
    const int kx = pi / N, ky = pi % N;
    const int mi = ((N - kx) % N) * N + (N - ky) % N;
    return HalfSpec<N, N * N * 8>{r, pi * 8, mi * 8};
}

// Elements per load chunk of the job multiply: at n = 32 with one pencil per
// lane, chunks of 4 keep the loop inside the 128-register cap; at n = 24 (nine
// waves per CU, registers to spare) half a pencil is read at once (measured
// best of 8, 12 and 24 in the batched kernel).  The other
// loops fence every 4 or 8 elements (QDVM_FENCE3).
template <int N, int Q>
constexpr int chunk3() { return (N == 32 && Q == 1) ? 4 : (N == 24 ? 12 : 8); }

#define QDVM_FENCE3(k)                                                                      \
    do {                                                                                    \
        if (((k) & (chunk3<N, Q>() == 4 ? 3 : 7)) == (chunk3<N, Q>() == 4 ? 3 : 7))          \
            __builtin_amdgcn_sched_barrier(0);                                              \
    } while (0)

// z = (alpha + i alpha') * spectrum for one job (spectral layout: lane pencil
// pi = Kx n + Ky, element k = Kz).  alpha(K) = D_M(e.K) - 1 walks one row of
// the LDS table (its argument advances by e_2 per element); alpha' is the job's
// FP64-built plane table.  The job weight is applied to the product (see
// job2d_multiply).
// C: elements per load chunk, each chunk's reads issued before their use; 4 or
// less: reads interleaved with their use, fenced every 4 or 8 elements (the
// near-equilibrium cell, which holds two transforms, uses chunks of 8).
template <int N, int T, int Q, int C = chunk3<N, Q>()>
__device__ __forceinline__ void job3d_multiply(float2 (&z)[Q][N], rsrc_t rs, const DevPlan& pl, const JobDesc& J,
                                               int jb, const float* atab, int tid)
{
    constexpr int NN = N * N, RS = NN * 4;
    const rsrc_t rap = make_rsrc(pl.aperp + (size_t)jb * NN * N, NN * N * 4);
    if constexpr (mirror_slabs<N, T>()) {
        // elements k and n - k together: the lane reads its own half pencil of the
        // spectrum and of the plane table; element n - k of its pencil is the
        // conjugate (for the even plane table: the value) of element k of the
        // mirror pencil (-Kx, -Ky), which a lane of the same wave has just read,
        // so it comes by shuffle.  The line multiplier walks forward for k and
        // backward (from k = n - 1) for n - k.
        const int pi = spec_pi<N, T>(tid), kx = pi / N, ky = pi % N;
        const int mlane = mirror_thread<N, T>(tid) & 63;
        const HalfSpec<N, N * N * 8> hs = half3d<N>(rs, pi);
        RowWalk<N> a(atab + J.M * N, modc<N>(J.e[0] * kx + J.e[1] * ky), modc<N>(J.e[2]));
        RowWalk<N> am(atab + J.M * N, modc<N>(J.e[0] * kx + J.e[1] * ky - J.e[2]), modc<N>(-J.e[2]));
        // the whole half pencil's reads in flight at once (the transform's registers
        // are free here): 1.60 against 1.63 ms per 2048 cells with chunks of 4
        constexpr int H = N / 2 + 1, CH = H;
#pragma unroll
        for (int k0 = 0; k0 < H; k0 += CH) {
            float2 F[CH];
            float a2[CH];
#pragma unroll
            for (int i = 0; i < CH; ++i)
                if (k0 + i < H) {
                    F[i] = hs.get(k0 + i);
                    a2[i] = bload(rap, pi * 4, (k0 + i) * RS);
                }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                const int k = k0 + i;
                if (k >= H) break;
                const float al = a.get();
                z[0][k] = make_float2(__builtin_fmaf(al, F[i].x, -a2[i] * F[i].y),
                                      __builtin_fmaf(al, F[i].y, a2[i] * F[i].x));
                a.next();
                if (k >= 1 && k < N / 2) {
                    const float2 Fm = make_float2(__shfl(F[i].x, mlane, 64), -__shfl(F[i].y, mlane, 64));
                    const float a2m = __shfl(a2[i], mlane, 64);
                    const float bl = am.get();
                    z[0][N - k] = make_float2(__builtin_fmaf(bl, Fm.x, -a2m * Fm.y),
                                              __builtin_fmaf(bl, Fm.y, a2m * Fm.x));
                    am.next();
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int pi = spec_pi<N, T>(tid + q * T), kx = pi / N, ky = pi % N;
        const HalfSpec<N, N * N * 8> hs = half3d<N>(rs, pi);
        RowWalk<N> a(atab + J.M * N, modc<N>(J.e[0] * kx + J.e[1] * ky), modc<N>(J.e[2]));
        if constexpr (C <= 4) {
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const float2 F = hs.get(k);
                const float al = a.get(), a2 = bload(rap, pi * 4, k * RS);
                z[q][k] = make_float2(__builtin_fmaf(al, F.x, -a2 * F.y), __builtin_fmaf(al, F.y, a2 * F.x));
                a.next();
                QDVM_FENCE3(k);
            }
        } else {
#pragma unroll
            for (int k0 = 0; k0 < N; k0 += C) {
                float2 F[C];
                float a2[C];
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    F[i] = hs.get(k0 + i);
                    a2[i] = bload(rap, pi * 4, (k0 + i) * RS);
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    const float al = a.get();
                    z[q][k0 + i] = make_float2(__builtin_fmaf(al, F[i].x, -a2[i] * F[i].y),
                                               __builtin_fmaf(al, F[i].y, a2[i] * F[i].x));
                    a.next();
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
}

// Jobs jb0, jb0 + jstep, ... of the direction loop; the loss only if `loss`
// (a cell whose jobs are spread over several workgroups: each writes its part).
// The last LACC elements of each lane's gain accumulator live in LDS (`lacc`,
// LACC x T*Q floats, each lane touching only its own words) instead of
// registers: at n = 32 with one pencil per lane the register cap would
// otherwise spill them to scratch memory around every job.
template <int N, int T, int RV, int LACC = 0>
__device__ __forceinline__ void cell3d_eval(const DevPlan& pl, const Cell3D& cl, rsrc_t rlam,
                                            const float* __restrict__ jobw, float dt, float* xb,
                                            const float* dtab, int tid, int jb0 = 0, int jstep = 1,
                                            bool loss = true, float* lacc = nullptr)
{
    constexpr int NN = N * N, Q = NN / T, RS = NN * 4, NR = N - LACC;
    float2 z[Q][N];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int x = 0; x < N; ++x) z[q][x] = make_float2(bload(cl.f, (tid + q * T) * 4, x * RS), 0.f);
    fwd3d<N, T, Q, RV>(z, xb, tid);
    float acc[Q][NR > 0 ? NR : 1];
    auto lslot = [&](int q, int x) -> float& { return lacc[(x - NR) * (T * Q) + tid + q * T]; };
#pragma unroll
    for (int q = 0; q < Q; ++q) half3d<N>(cl.fh, spec_pi<N, T>(tid + q * T)).put(z[q]);
    if (loss) {
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int k0 = 0; k0 < N; k0 += 8) {
                float l[8];
                load_run<8>(l, rlam, spec_pi<N, T>(tid + q * T) * 4, k0, RS);
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    z[q][k0 + k].x *= l[k];
                    z[q][k0 + k].y *= l[k];
                }
            }
        inv3d<N, T, Q, RV>(z, xb, tid);
        constexpr int C = N % 8 == 0 ? 8 : N;
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int x0 = 0; x0 < N; x0 += C) {
                float fv[C];
                load_run<C>(fv, cl.f, (tid + q * T) * 4, x0, RS);
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    const int x = x0 + i;
                    const float v = -fv[i] * z[q][x].x;
                    if (x < NR) acc[q][x] = v;
                    else lslot(q, x) = v;
                }
            }
    } else {
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int k = 0; k < N; ++k) {
                if (k < NR) acc[q][k] = 0.f;
                else lslot(q, k) = 0.f;
            }
    }
    // the jobs read mirrored pencils of the spectrum, written by other threads
    __syncthreads();

    const float* atab = dtab_alpha(dtab, pl);
    for (int jb = jb0; jb < pl.njobs; jb += jstep) {
        const JobDesc J = gload(pl.jobs, jb);
        const float cw = gload(jobw, jb);
        job3d_multiply<N, T, Q>(z, cl.fh, pl, J, jb, atab, tid);
        inv3d<N, T, Q, RV>(z, xb, tid);
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int x = 0; x < N; ++x) {
                if (x < NR) acc[q][x] = __builtin_fmaf(cw * z[q][x].x, z[q][x].y, acc[q][x]);
                else lslot(q, x) = __builtin_fmaf(cw * z[q][x].x, z[q][x].y, lslot(q, x));
            }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int v = (tid + q * T) * 4;
        if (dt == 0.f) {
#pragma unroll
            for (int x = 0; x < N; ++x) bstore(x < NR ? acc[q][x] : lslot(q, x), cl.q, v, x * RS);
        } else {
            float fv[N];
            load_run<N>(fv, cl.f, v, 0, RS);
#pragma unroll
            for (int x = 0; x < N; ++x)
                bstore(__builtin_fmaf(dt, x < NR ? acc[q][x] : lslot(q, x), fv[x]), cl.q, v, x * RS);
        }
    }
}


// z = alpha ghat + i alpha' fhat for one direction of the bilinear operator
// (spectral layout as job3d_multiply; chunks of C elements, each chunk's reads
// issued before their use).
template <int N, int T, int Q, int C>
__device__ __forceinline__ void job3d_multiply_bilinear(float2 (&z)[Q][N], rsrc_t rgs, rsrc_t rfs, const DevPlan& pl,
                                                        const JobDesc& J, int jb, const float* atab, int tid)
{
    constexpr int NN = N * N, RS = NN * 4;
    const rsrc_t rap = make_rsrc(pl.aperp + (size_t)jb * NN * N, NN * N * 4);
    if constexpr (mirror_slabs<N, T>()) {
        // elements k and n - k together, the mirror halves of both spectra and of
        // the plane table by shuffle (as in job3d_multiply)
        const int pi = spec_pi<N, T>(tid), kx = pi / N, ky = pi % N;
        const int mlane = mirror_thread<N, T>(tid) & 63;
        const HalfSpec<N, N * N * 8> gs = half3d<N>(rgs, pi);
        const HalfSpec<N, N * N * 8> fs = half3d<N>(rfs, pi);
        RowWalk<N> a(atab + J.M * N, modc<N>(J.e[0] * kx + J.e[1] * ky), modc<N>(J.e[2]));
        RowWalk<N> am(atab + J.M * N, modc<N>(J.e[0] * kx + J.e[1] * ky - J.e[2]), modc<N>(-J.e[2]));
        constexpr int H = N / 2 + 1;
#pragma unroll
        for (int k0 = 0; k0 < H; k0 += C) {
            float2 G[C], F[C];
            float a2[C];
#pragma unroll
            for (int i = 0; i < C; ++i)
                if (k0 + i < H) {
                    G[i] = gs.get(k0 + i);
                    F[i] = fs.get(k0 + i);
                    a2[i] = bload(rap, pi * 4, (k0 + i) * RS);
                }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < C; ++i) {
                const int k = k0 + i;
                if (k >= H) break;
                const float al = a.get();
                z[0][k] = make_float2(__builtin_fmaf(al, G[i].x, -a2[i] * F[i].y),
                                      __builtin_fmaf(al, G[i].y, a2[i] * F[i].x));
                a.next();
                if (k >= 1 && k < N / 2) {
                    const float2 Gm = make_float2(__shfl(G[i].x, mlane, 64), -__shfl(G[i].y, mlane, 64));
                    const float2 Fm = make_float2(__shfl(F[i].x, mlane, 64), -__shfl(F[i].y, mlane, 64));
                    const float a2m = __shfl(a2[i], mlane, 64);
                    const float bl = am.get();
                    z[0][N - k] = make_float2(__builtin_fmaf(bl, Gm.x, -a2m * Fm.y),
                                              __builtin_fmaf(bl, Gm.y, a2m * Fm.x));
                    am.next();
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int pi = spec_pi<N, T>(tid + q * T), kx = pi / N, ky = pi % N;
        const HalfSpec<N, N * N * 8> gs = half3d<N>(rgs, pi);
        const HalfSpec<N, N * N * 8> fs = half3d<N>(rfs, pi);
        RowWalk<N> a(atab + J.M * N, modc<N>(J.e[0] * kx + J.e[1] * ky), modc<N>(J.e[2]));
#pragma unroll
        for (int k0 = 0; k0 < N; k0 += C) {
            float2 G[C], F[C];
            float a2[C];
#pragma unroll
            for (int i = 0; i < C; ++i) {
                G[i] = gs.get(k0 + i);
                F[i] = fs.get(k0 + i);
                a2[i] = bload(rap, pi * 4, (k0 + i) * RS);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < C; ++i) {
                const float al = a.get();
                z[q][k0 + i] = make_float2(__builtin_fmaf(al, G[i].x, -a2[i] * F[i].y),
                                           __builtin_fmaf(al, G[i].y, a2[i] * F[i].x));
                a.next();
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// Bilinear operator Q(g, f) of one 3D cell (see cell2d_eval_bilinear): the
// transforms of g and f as half spectra in rgh and cl.fh, one inverse
// transform of alpha_p ghat + i alpha'_p fhat per direction, loss
// -g IFFT(Lambda fhat).  cl.f holds f, rg holds g; the Euler form updates g.
// dirw: per-direction weights / n^6.  LACC as in cell3d_eval.
template <int N, int T, int RV, int LACC = 0>
__device__ __forceinline__ void cell3d_eval_bilinear(const DevPlan& pl, const Cell3D& cl, rsrc_t rg, rsrc_t rgh,
                                                     rsrc_t rlam, const float* __restrict__ dirw, float dt,
                                                     float* xb, const float* dtab, int tid, float* lacc)
{
    constexpr int NN = N * N, Q = NN / T, RS = NN * 4, NR = N - LACC;
    float2 z[Q][N];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int x = 0; x < N; ++x) z[q][x] = make_float2(bload(rg, (tid + q * T) * 4, x * RS), 0.f);
    fwd3d<N, T, Q, RV>(z, xb, tid);
#pragma unroll
    for (int q = 0; q < Q; ++q) half3d<N>(rgh, spec_pi<N, T>(tid + q * T)).put(z[q]);
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int x = 0; x < N; ++x) z[q][x] = make_float2(bload(cl.f, (tid + q * T) * 4, x * RS), 0.f);
    fwd3d<N, T, Q, RV>(z, xb, tid);
#pragma unroll
    for (int q = 0; q < Q; ++q) half3d<N>(cl.fh, spec_pi<N, T>(tid + q * T)).put(z[q]);
    float acc[Q][NR > 0 ? NR : 1];
    auto lslot = [&](int q, int x) -> float& { return lacc[(x - NR) * (T * Q) + tid + q * T]; };
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int k0 = 0; k0 < N; k0 += 8) {
            float l[8];
            load_run<8>(l, rlam, spec_pi<N, T>(tid + q * T) * 4, k0, RS);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                z[q][k0 + k].x *= l[k];
                z[q][k0 + k].y *= l[k];
            }
        }
    inv3d<N, T, Q, RV>(z, xb, tid);
    {
        constexpr int C = N % 8 == 0 ? 8 : N;
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int x0 = 0; x0 < N; x0 += C) {
                float gv[C];
                load_run<C>(gv, rg, (tid + q * T) * 4, x0, RS);
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    const int x = x0 + i;
                    const float v = -gv[i] * z[q][x].x;
                    if (x < NR) acc[q][x] = v;
                    else lslot(q, x) = v;
                }
            }
    }
    // the directions read mirrored pencils of both spectra, written by other threads
    __syncthreads();

    const float* atab = dtab_alpha(dtab, pl);
    for (int jb = 0; jb < pl.njobs; ++jb) {
        const JobDesc J = gload(pl.jobs, jb);
        const float cw = gload(dirw, J.p);
        job3d_multiply_bilinear<N, T, Q, (N == 32 && Q == 1) ? 4 : 8>(z, rgh, cl.fh, pl, J, jb, atab, tid);
        inv3d<N, T, Q, RV>(z, xb, tid);
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int x = 0; x < N; ++x) {
                if (x < NR) acc[q][x] = __builtin_fmaf(cw * z[q][x].x, z[q][x].y, acc[q][x]);
                else lslot(q, x) = __builtin_fmaf(cw * z[q][x].x, z[q][x].y, lslot(q, x));
            }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int v = (tid + q * T) * 4;
        if (dt == 0.f) {
#pragma unroll
            for (int x = 0; x < N; ++x) bstore(x < NR ? acc[q][x] : lslot(q, x), cl.q, v, x * RS);
        } else {
            float gv[N];
            load_run<N>(gv, rg, v, 0, RS);
#pragma unroll
            for (int x = 0; x < N; ++x)
                bstore(__builtin_fmaf(dt, x < NR ? acc[q][x] : lslot(q, x), gv[x]), cl.q, v, x * RS);
        }
    }
}


// Block-wide sum of five doubles (moments); every thread gets the totals.
template <int T>
__device__ __forceinline__ void block_sum5d(double (&v)[5], double* red, int tid)
{
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
    __syncthreads();
    if ((tid & 63) == 0)
#pragma unroll
        for (int k = 0; k < 5; ++k) red[(tid >> 6) * 5 + k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < (T + 63) / 64; ++w) t += red[w * 5 + k];
        v[k] = t;
    }
}

// Near-equilibrium evaluation of one 3D cell: Q(f, f) - Q(M, M) through
// Q(g, f) + Q(M, g), g = f - M, M the Maxwellian of the cell's moments (the
// transform layout, the error argument and STAGE are those of
// cell2d_eval_split).
template <int N, int T, int RV, bool STAGE>
__device__ __forceinline__ void cell3d_eval_split(const DevPlan& pl, const Cell3D& cl, rsrc_t rgh, rsrc_t rtg,
                                                  rsrc_t rlam, const float* __restrict__ jobw, float dt, float* xb,
                                                  double* red, const float* dtab, int tid)
{
    constexpr int NN = N * N, Q = NN / T, RS = NN * 4, RS2 = NN * 8;
    double mom[5] = {0.0, 0.0, 0.0, 0.0, 0.0};   // sum f, sum x f, sum y f, sum z f, sum |x|^2 f
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int pi = tid + q * T, py = pi / N, pz = pi % N;
        double ps = 0.0;
#pragma unroll
        for (int x0 = 0; x0 < N; x0 += 8) {
            float fv[8];
            load_run<8>(fv, cl.f, pi * 4, x0, RS);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const double v = fv[i];
                ps += v;
                mom[1] += (double)(x0 + i) * v;
                mom[4] += (double)((x0 + i) * (x0 + i)) * v;
            }
        }
        mom[0] += ps;
        mom[2] += (double)py * ps;
        mom[3] += (double)pz * ps;
        mom[4] += (double)(py * py + pz * pz) * ps;
    }
    block_sum5d<T>(mom, red, tid);
    const double s0 = mom[0];
    const double mx = mom[1] / s0, my = mom[2] / s0, mz = mom[3] / s0;
    const double var = (mom[4] / s0 - mx * mx - my * my - mz * mz) / 3.0;
    const bool ok = s0 > 0.0 && var > 0.25 && __builtin_isfinite(var) && __builtin_isfinite(mx) &&
                    __builtin_isfinite(my) && __builtin_isfinite(mz);
    const double inv2v = ok ? 0.5 / var : 0.0;
    const double C = ok ? s0 / ((2.0 * kPi * var) * sqrt(2.0 * kPi * var)) : 0.0;
    // M(x, y, z) = eyz(y, z) ex(x): the n factors ex(x) sit in LDS after the
    // reduction slots of block_sum5d (5 doubles per wave)
    double* ex = red + 5 * ((T + 63) / 64);
    if (tid < N) ex[tid] = ok ? exp(-(tid - mx) * (tid - mx) * inv2v) : 0.0;
    double eyz[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int pi = tid + q * T, py = pi / N, pz = pi % N;
        eyz[q] = ok ? C * exp(-((py - my) * (py - my) + (pz - mz) * (pz - mz)) * inv2v) : 0.0;
    }
    __syncthreads();

    float2 z[Q][N];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int x0 = 0; x0 < N; x0 += 8) {
            float fv[8];
            double e[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) e[i] = ex[x0 + i];
            load_run<8>(fv, cl.f, (tid + q * T) * 4, x0, RS);
#pragma unroll
            for (int i = 0; i < 8; ++i) z[q][x0 + i] = make_float2((float)((double)fv[i] - eyz[q] * e[i]), 0.f);
        }
    fwd3d<N, T, Q, RV>(z, xb, tid);
#pragma unroll
    for (int q = 0; q < Q; ++q) half3d<N>(rgh, spec_pi<N, T>(tid + q * T)).put(z[q]);
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int k0 = 0; k0 < N; k0 += 8) {
            float l[8];
            load_run<8>(l, rlam, spec_pi<N, T>(tid + q * T) * 4, k0, RS);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                z[q][k0 + k].x *= l[k];
                z[q][k0 + k].y *= l[k];
            }
        }
    inv3d<N, T, Q, RV>(z, xb, tid);             // l(g)
    float acc[Q][N];                            // holds l(g) until l(f) is formed
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int x = 0; x < N; ++x) acc[q][x] = z[q][x].x;
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int x = 0; x < N; ++x) z[q][x] = make_float2(bload(cl.f, (tid + q * T) * 4, x * RS), 0.f);
    fwd3d<N, T, Q, RV>(z, xb, tid);
#pragma unroll
    for (int q = 0; q < Q; ++q) half3d<N>(cl.fh, spec_pi<N, T>(tid + q * T)).put(z[q]);
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int k0 = 0; k0 < N; k0 += 8) {
            float l[8];
            load_run<8>(l, rlam, spec_pi<N, T>(tid + q * T) * 4, k0, RS);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                z[q][k0 + k].x *= l[k];
                z[q][k0 + k].y *= l[k];
            }
        }
    inv3d<N, T, Q, RV>(z, xb, tid);             // l(f)
    {
        // M again from the LDS factors (read after the barriers of the transforms)
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int x0 = 0; x0 < N; x0 += 8) {
                float fv[8];
                double e[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) e[i] = ex[x0 + i];
                load_run<8>(fv, cl.f, (tid + q * T) * 4, x0, RS);
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int x = x0 + i;
                    const double m = eyz[q] * e[i];
                    const float g = (float)((double)fv[i] - m);
                    acc[q][x] = -__builtin_fmaf(g, z[q][x].x, (float)m * acc[q][x]);
                }
            }
    }

    const float* atab = dtab_alpha(dtab, pl);
    for (int jb = 0; jb < pl.njobs; ++jb) {
        const JobDesc J = gload(pl.jobs, jb);
        const float cw = gload(jobw, jb);
        float2 tg[Q][N];
        job3d_multiply<N, T, Q, (chunk3<N, Q>() == 4 ? 4 : 8)>(tg, rgh, pl, J, jb, atab, tid);
        inv3d<N, T, Q, RV>(tg, xb, tid);         // line(g) + i plane(g)
        if constexpr (STAGE) {
#pragma unroll
            for (int q = 0; q < Q; ++q)
#pragma unroll
                for (int x = 0; x < N; ++x) bstore2(tg[q][x], rtg, (tid + q * T) * 8, x * RS2);
        }
        job3d_multiply<N, T, Q, (chunk3<N, Q>() == 4 ? 4 : 8)>(z, cl.fh, pl, J, jb, atab, tid);
        inv3d<N, T, Q, RV>(z, xb, tid);          // line(f) + i plane(f)
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int x0 = 0; x0 < N; x0 += 8) {
                float2 t[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) t[i] = STAGE ? bload2(rtg, (tid + q * T) * 8, (x0 + i) * RS2) : tg[q][x0 + i];
                if constexpr (STAGE) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int x = x0 + i;
                    const float gain = __builtin_fmaf(t[i].x, z[q][x].y, (z[q][x].x - t[i].x) * t[i].y);
                    acc[q][x] = __builtin_fmaf(cw, gain, acc[q][x]);
                }
            }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int v = (tid + q * T) * 4;
        if (dt == 0.f) {
#pragma unroll
            for (int x = 0; x < N; ++x) bstore(acc[q][x], cl.q, v, x * RS);
        } else {
            float fv[N];
            load_run<N>(fv, cl.f, v, 0, RS);
#pragma unroll
            for (int x = 0; x < N; ++x) bstore(__builtin_fmaf(dt, acc[q][x], fv[x]), cl.q, v, x * RS);
        }
    }
}

// um[q][r] = z of the mirror pencil (-Kx, -Ky) at element (n - r) mod n, i.e.
// uhat(-K) for K = (Kx, Ky, r), r = 0..n/2, through the LDS cube (real parts,
// then imaginary parts; each lane writes the elements its mirror lane needs).
template <int N, int T, int Q>
__device__ __forceinline__ void mirror_exchange(const float2 (&z)[Q][N], float2 (&um)[Q][N / 2 + 1], float* xb,
                                                int tid)
{
    constexpr int NN = N * N;
    if constexpr (mirror_slabs<N, T>()) {
        // the mirror pencil is in the same wave: shuffles, no LDS round trip
        const int mlane = mirror_thread<N, T>(tid) & 63;
#pragma unroll
        for (int r = 0; r <= N / 2; ++r) {
            const float2 v = z[0][(N - r) % N];
            um[0][r] = make_float2(__shfl(v.x, mlane, 64), __shfl(v.y, mlane, 64));
        }
        return;
    }
#pragma unroll
    for (int part = 0; part < 2; ++part) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int r = 0; r <= N / 2; ++r) {
                const float2 v = z[q][(N - r) % N];
                xb[r * NN + tid + q * T] = part ? v.y : v.x;
            }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int mi = mirror_thread<N, T>(tid + q * T);
#pragma unroll
            for (int r = 0; r <= N / 2; ++r) {
                const float v = xb[r * NN + mi];
                if (part) um[q][r].y = v;
                else um[q][r].x = v;
            }
        }
    }
}

// Adjoint of one cell.  With c the cotangent and unnormalised transforms F:
//   l + i C(cf) = IFFT(Lambda (fhat + i F(cf)))            (both real)
//   per job:  u + i v = IFFT((a + i a') fhat) = n^d (g + i h)
//             dQ/dw_j part: <c, g h> - <cf, l_j>, the second term by Parseval:
//             n^{-2d} sum_x c u v - n^{-d} sum_K a a' R(K),
//             R = Re(conj(F(cf)) fhat)  (real and even: stored as half pencils)
//             S += W_j / n^{2d} (a - i a') F(c v + i c u)
//   grad_f = Re IFFT(S) - c l - C(cf)
// which uses A(c h) + B(c g) = Re IFFT((a - i a') F(c h + i c g)), valid because
// the multipliers a = alpha_j and a' = alpha'_j are real and even.
// Jobs jb0, jb0 + jstep, ...; the loss part only if `loss` (see cell3d_eval).
// rr: R of the cell (half pencils, 4 bytes per element); rnone: a descriptor of
// the accumulator's base with extent 0.
template <int N, int T, int RV>
__device__ __forceinline__ void cell3d_vjp(const DevPlan& pl, const Cell3D& cl, rsrc_t rc, rsrc_t rr,
                                           rsrc_t rsh, rsrc_t rnone, rsrc_t rlam, const float* __restrict__ jobw,
                                           double* __restrict__ gwp, bool gw_first, float inv_n2, float inv_n,
                                           float* xb, float* red, const float* dtab, int tid, int jb0 = 0,
                                           int jstep = 1, bool loss = true)
{
    constexpr int NN = N * N, Q = NN / T, RS = NN * 4, RS2 = NN * 8;
    float2 z[Q][N];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int x = 0; x < N; ++x) z[q][x] = make_float2(bload(cl.f, (tid + q * T) * 4, x * RS), 0.f);
    fwd3d<N, T, Q, RV>(z, xb, tid);
#pragma unroll
    for (int q = 0; q < Q; ++q) half3d<N>(cl.fh, spec_pi<N, T>(tid + q * T)).put(z[q]);
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int x = 0; x < N; ++x) {
            const int v = (tid + q * T) * 4;
            z[q][x] = make_float2(bload(rc, v, x * RS) * bload(cl.f, v, x * RS), 0.f);
            QDVM_FENCE3(x);
        }
    fwd3d<N, T, Q, RV>(z, xb, tid);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int pi = spec_pi<N, T>(tid + q * T);
        const HalfSpec<N, N * N * 8> fh = half3d<N>(cl.fh, pi);
        // own half of the pencil, written by this lane; each chunk's reads are
        // issued before its stores (which the compiler cannot tell apart from them)
#pragma unroll
        for (int k0 = 0; k0 <= N / 2; k0 += 4) {
            float2 F[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (k0 + i <= N / 2) F[i] = fh.get(k0 + i);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (k0 + i <= N / 2)
                    bstore(__builtin_fmaf(z[q][k0 + i].x, F[i].x, z[q][k0 + i].y * F[i].y), rr, pi * 4,
                           (k0 + i) * RS);
        }
    }
    if (loss) {
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const int pi = spec_pi<N, T>(tid + q * T);
                const float2 F = half3d<N>(cl.fh, pi).get(k);
                const float l = bload(rlam, pi * 4, k * RS);
                z[q][k] = make_float2(l * (F.x - z[q][k].y), l * (F.y + z[q][k].x));
                QDVM_FENCE3(k);
            }
        inv3d<N, T, Q, RV>(z, xb, tid);
        // -c l - C(cf) goes to grad_f now and is completed after the direction
        // loop, so that no pencil-sized accumulator stays live through it
        constexpr int C = N % 8 == 0 ? 8 : N;
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int x0 = 0; x0 < N; x0 += C) {
                const int v = (tid + q * T) * 4;
                float cv[C];
                load_run<C>(cv, rc, v, x0, RS);
#pragma unroll
                for (int i = 0; i < C; ++i)
                    bstore(-cv[i] * z[q][x0 + i].x - z[q][x0 + i].y, cl.q, v, (x0 + i) * RS);
            }
    } else {
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int k = 0; k < N; ++k) bstore(0.f, cl.q, (tid + q * T) * 4, k * RS);
    }
    // the jobs read mirrored pencils of the spectrum and of R, written by other threads
    __syncthreads();

    // The accumulator S lives in memory between jobs, in half pencils.  The
    // first job reads it through an empty descriptor (every read returns 0 and
    // every write is dropped, with no memory request), so it needs no zero fill.
    // When the mirror pencil is in the same wave the last job keeps its sums in
    // z, the final transform's input, and writes through the empty descriptor
    // instead of storing them to be read back.
    constexpr bool keep_last = mirror_slabs<N, T>();
    const float* atab = dtab_alpha(dtab, pl);
    for (int jb = jb0; jb < pl.njobs; jb += jstep) {
        const JobDesc J = gload(pl.jobs, jb);
        const float cw = gload(jobw, jb);
        const rsrc_t rsr = jb == jb0 ? rnone : rsh;
        const rsrc_t rsw = keep_last && jb + jstep >= pl.njobs ? rnone : rsh;
        const rsrc_t rap = make_rsrc(pl.aperp + (size_t)jb * NN * N, NN * N * 4);
        float spart = 0.f;
        if constexpr (mirror_slabs<N, T>()) {
            // elements k and n - k together: the mirror halves of the spectrum, of R
            // (even) and of the plane table (even) by shuffle (as in job3d_multiply)
            const int pi = spec_pi<N, T>(tid), kx = pi / N, ky = pi % N;
            const int mlane = mirror_thread<N, T>(tid) & 63;
            const HalfSpec<N, N * N * 8> fh = half3d<N>(cl.fh, pi);
            RowWalk<N> a(atab + J.M * N, modc<N>(J.e[0] * kx + J.e[1] * ky), modc<N>(J.e[2]));
            RowWalk<N> am(atab + J.M * N, modc<N>(J.e[0] * kx + J.e[1] * ky - J.e[2]), modc<N>(-J.e[2]));
            constexpr int H = N / 2 + 1, CH = 4;
#pragma unroll
            for (int k0 = 0; k0 < H; k0 += CH) {
                float2 F[CH];
                float R[CH], a2[CH];
#pragma unroll
                for (int i = 0; i < CH; ++i)
                    if (k0 + i < H) {
                        F[i] = fh.get(k0 + i);
                        R[i] = bload(rr, pi * 4, (k0 + i) * RS);
                        a2[i] = bload(rap, pi * 4, (k0 + i) * RS);
                    }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const int k = k0 + i;
                    if (k >= H) break;
                    const float al = a.get();
                    z[0][k] = make_float2(__builtin_fmaf(al, F[i].x, -a2[i] * F[i].y),
                                          __builtin_fmaf(al, F[i].y, a2[i] * F[i].x));
                    spart = __builtin_fmaf(al * a2[i], R[i], spart);
                    a.next();
                    if (k >= 1 && k < N / 2) {
                        const float2 Fm = make_float2(__shfl(F[i].x, mlane, 64), -__shfl(F[i].y, mlane, 64));
                        const float Rm = __shfl(R[i], mlane, 64), a2m = __shfl(a2[i], mlane, 64);
                        const float bl = am.get();
                        z[0][N - k] = make_float2(__builtin_fmaf(bl, Fm.x, -a2m * Fm.y),
                                                  __builtin_fmaf(bl, Fm.y, a2m * Fm.x));
                        spart = __builtin_fmaf(bl * a2m, Rm, spart);
                        am.next();
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
#pragma unroll
        for (int q = 0; q < (mirror_slabs<N, T>() ? 0 : Q); ++q) {
            const int pi = spec_pi<N, T>(tid + q * T), kx = pi / N, ky = pi % N;
            const HalfSpec<N, N * N * 8> fh = half3d<N>(cl.fh, pi);
            const int rown = pi * 4, rmir = fh.mir / 2;
            RowWalk<N> a(atab + J.M * N, modc<N>(J.e[0] * kx + J.e[1] * ky), modc<N>(J.e[2]));
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const float2 F = fh.get(k);
                const float R = k <= N / 2 ? bload(rr, rown, k * RS) : bload(rr, rmir, (N - k) * RS);
                const float al = a.get(), a2 = bload(rap, pi * 4, k * RS);
                z[q][k] = make_float2(__builtin_fmaf(al, F.x, -a2 * F.y), __builtin_fmaf(al, F.y, a2 * F.x));
                spart = __builtin_fmaf(al * a2, R, spart);
                a.next();
                QDVM_FENCE3(k);
            }
        }
        inv3d<N, T, Q, RV>(z, xb, tid);
        float rpart = 0.f;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int v = reread((tid + q * T) * 4);
#pragma unroll
            for (int x = 0; x < N; ++x) {
                const float c = bload(rc, v, x * RS);
                rpart = __builtin_fmaf(c * z[q][x].x, z[q][x].y, rpart);
                z[q][x] = make_float2(c * z[q][x].y, c * z[q][x].x);
                // the cotangent's reads in flight 16 at a time (0.205 -> 0.202 ms for
                // the adjoint of 64 n = 32 cells against the transform-sized fences)
                if ((x & 15) == 15) __builtin_amdgcn_sched_barrier(0);
            }
        }
        const double tot = block_sumd<T>((double)rpart * inv_n2 - (double)spart * inv_n,
                                         reinterpret_cast<double*>(red), tid);
        if (tid == 0) gw_accumulate(gwp + jb, tot, gw_first);
        fwd3d<N, T, Q, RV>(z, xb, tid);
        // Only the Hermitian part of (a - i a') uhat reaches Re IFFT(S), so S is
        // kept as that part, in half pencils: it needs uhat(-K), held by the
        // mirror lane and exchanged through LDS.
        float2 um[Q][N / 2 + 1];
        mirror_exchange<N, T, Q>(z, um, xb, tid);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            // the multipliers are read again rather than kept from the first
            // multiply: holding them through two transforms would spill
            const int pi = spec_pi<N, T>(reread(tid + q * T)), kx = pi / N, ky = pi % N;
            RowWalk<N> a(atab + J.M * N, modc<N>(J.e[0] * kx + J.e[1] * ky), modc<N>(J.e[2]));
#pragma unroll
            for (int k0 = 0; k0 <= N / 2; k0 += 4) {
                // the chunk's reads go out before its stores (the compiler would
                // otherwise wait for each accumulator read in turn)
                float2 sv[4];
                float a2[4], a1[4];
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (k0 + i <= N / 2) {
                        sv[i] = bload2(rsr, pi * 8, (k0 + i) * RS2);
                        a2[i] = 0.5f * cw * bload(rap, pi * 4, (k0 + i) * RS);
                        a1[i] = 0.5f * cw * a.get();
                        a.next();
                    }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int k = k0 + i;
                    if (k > N / 2) break;
                    const float al = a1[i];
                    // (a/2)(u + conj m) - i (a'/2)(u - conj m), m = uhat(-K)
                    const float2 u = z[q][k], m = um[q][k];
                    float2 t = make_float2(__builtin_fmaf(al, u.x + m.x, a2[i] * (u.y + m.y)),
                                           __builtin_fmaf(al, u.y - m.y, -a2[i] * (u.x - m.x)));
                    const float2 sum = make_float2(t.x + sv[i].x, t.y + sv[i].y);
                    if constexpr (keep_last) z[q][k] = sum;   // u = z[q][k] is not read again in this job
                    bstore2(sum, rsw, pi * 8, k * RS2);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    if (jb0 < pl.njobs) {
        if constexpr (keep_last) {
            // z[0][0..n/2] holds the own half pencil of S; element k > n/2 is the
            // conjugate of element n - k of the mirror pencil (-Kx, -Ky)
            const int mlane = mirror_thread<N, T>(tid) & 63;
#pragma unroll
            for (int k = N / 2 + 1; k < N; ++k)
                z[0][k] = make_float2(__shfl(z[0][N - k].x, mlane, 64), -__shfl(z[0][N - k].y, mlane, 64));
        } else {
            // the other half of each pencil is the mirror lane's
            __syncthreads();
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const HalfSpec<N, N * N * 8> sh = half3d<N>(rsh, spec_pi<N, T>(tid + q * T));
#pragma unroll
                for (int k = 0; k < N; ++k) z[q][k] = sh.get(k);
            }
        }
        inv3d<N, T, Q, RV>(z, xb, tid);
        constexpr int C = N % 8 == 0 ? 8 : N;
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int x0 = 0; x0 < N; x0 += C) {
                const int v = (tid + q * T) * 4;
                float gv[C];
                load_run<C>(gv, cl.q, v, x0, RS);
#pragma unroll
                for (int i = 0; i < C; ++i) bstore(gv[i] + z[q][x0 + i].x, cl.q, v, (x0 + i) * RS);
            }
    }
}

}  // namespace qdvm
