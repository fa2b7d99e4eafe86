// Device code of one 2D cell of the fast DVM collision operator (included by
// the uniform-batch and the heterogeneous-batch kernels).
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
#pragma once
#include "kernels_common.h"

namespace qdvm {

// Lane j of an n-lane group holds row j of an n x n matrix; afterwards it holds
// row j of the transpose.  Row stride n+1 keeps both phases bank-conflict free.
template <int N>
__device__ __forceinline__ void group_transpose(float2 (&z)[N], float* xb, int j)
{
    wave_sync();
#pragma unroll
    for (int c = 0; c < N; ++c) xb[j * (N + 1) + c] = z[c].x;
    wave_sync();
#pragma unroll
    for (int c = 0; c < N; ++c) z[c].x = xb[c * (N + 1) + j];
    wave_sync();
#pragma unroll
    for (int c = 0; c < N; ++c) xb[j * (N + 1) + c] = z[c].y;
    wave_sync();
#pragma unroll
    for (int c = 0; c < N; ++c) z[c].y = xb[c * (N + 1) + j];
}

template <int N, int RV>
__device__ __forceinline__ void fwd2d(float2 (&z)[N], float* xb, int j)
{
    fftp<N, RV, -1>(z);
    group_transpose<N>(z, xb, j);
    fftp<N, RV, -1>(z);
}

template <int N, int RV>
__device__ __forceinline__ void inv2d(float2 (&z)[N], float* xb, int j)
{
    fftp<N, RV, 1>(z);
    group_transpose<N>(z, xb, j);
    fftp<N, RV, 1>(z);
}

// Buffers of one workgroup item (cpb consecutive cells).
struct Item2D {
    rsrc_t f, q, fh;     // cell data and the block's spectral scratch
    int vcell;           // byte offset of this lane's pencil in cell arrays (float)
    int vspec;           // byte offset of this lane's pencil in spectral arrays (float2)
};

// Half-stored spectrum of one 2D cell slot at the lane's row K0 = j (mirror row -j).
template <int N>
__device__ __forceinline__ HalfSpec<N, N * 8> half2d(rsrc_t r, int vspec, int j)
{
    return HalfSpec<N, N * 8>{r, vspec, vspec + ((((N - j) & (N - 1)) - j) * 8)};
}

// z = (alpha + i alpha') * spectrum for one job, the spectrum read from the
// slot rs at the lane's pencil.  alpha(K) = D_M(e.K) - 1 and alpha'(K) =
// D_M(e_perp.K) walk one row each of the LDS tables: along the lane's row
// K0 = j their arguments advance by e_1 and e_0 per element (K1).  (The job
// weight is applied to the product, not folded into alpha: the real and
// imaginary parts of one complex transform must be of the same size, or the
// rounding of the larger one swamps the smaller.)
// C > 0: the spectrum is read in chunks of C elements, each chunk's reads issued
// before any of them is used (for code whose register budget would otherwise
// lead the scheduler to wait for each read in turn); C = 0: reads interleaved
// with their use, fenced every 8 elements.
template <int N, int C = 0>
__device__ __forceinline__ void job2d_multiply(float2 (&z)[N], const HalfSpec<N, N * 8>& hs, const JobDesc& J,
                                               const float* dtab, const float* atab, int j)
{
    RowWalk<N> a(atab + J.M * N, modc<N>(J.e[0] * j), modc<N>(J.e[1]));
    RowWalk<N> b(dtab + J.M * N, modc<N>(-J.e[1] * j), modc<N>(J.e[0]));
    if constexpr (C == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const float2 F = hs.get(k);
            const float al = a.get(), ap = b.get();
            z[k] = make_float2(__builtin_fmaf(al, F.x, -ap * F.y), __builtin_fmaf(al, F.y, ap * F.x));
            a.next();
            b.next();
            QDVM_CHUNK_FENCE(k);
        }
    } else {
#pragma unroll
        for (int k0 = 0; k0 < N; k0 += C) {
            float2 F[C];
#pragma unroll
            for (int i = 0; i < C; ++i) F[i] = hs.get(k0 + i);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < C; ++i) {
                const float al = a.get(), ap = b.get();
                z[k0 + i] = make_float2(__builtin_fmaf(al, F[i].x, -ap * F[i].y),
                                        __builtin_fmaf(al, F[i].y, ap * F[i].x));
                a.next();
                b.next();
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// Gain accumulation over many jobs: the accumulator passes through values of
// the size of the gain and loss terms (several times |Q|), and adding one
// rounded product per job lets FP32 rounding grow with the number of jobs
// (at 44 and 128 jobs it reaches 1e-5 of max|Q|).  With a sum buffer `rsc`
// (per element a float pair: sum S, compensation C, at the spectral slot's
// offsets), the accumulator is flushed every kFlushJobs jobs into S by
// compensated (Kahan) addition and restarts from zero, so each FP32 partial
// sum holds at most kFlushJobs (qdvm_internal.h) products; the result is S - C.

template <int N>
__device__ __forceinline__ void flush_gain(float (&acc)[N], rsrc_t rsc, int vspec, bool first)
{
    constexpr int RS2 = N * 8, C = N < 16 ? N : 16;
#pragma unroll
    for (int i0 = 0; i0 < N; i0 += C) {
        float2 sc[C];
        if (!first) {
#pragma unroll
            for (int i = 0; i < C; ++i) sc[i] = bload2(rsc, vspec, (i0 + i) * RS2);
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int i = 0; i < C; ++i) {
            float2 v;
            if (first) {
                v = make_float2(acc[i0 + i], 0.f);
            } else {
                const float y = acc[i0 + i] - sc[i].y;
                const float t = sc[i].x + y;
                v = make_float2(t, (t - sc[i].x) - y);
            }
            bstore2(v, rsc, vspec, (i0 + i) * RS2);
            acc[i0 + i] = 0.f;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// rsc: the sum buffer of the flushed accumulation (used when flush is set,
// i.e. when the plan has more than kFlushJobs jobs).
// Per-job multiplier tables (JT launches).  Lane j of a 2D cell reads a row
// of multipliers at (s_j + d k) mod n for k = 0..n-1: the line multiplier at
// e.K (s_j = e0 j, d = e1) and the plane multiplier at e_perp.K (s_j = -e1 j,
// d = e0).  With g = gcd(d, n), L = n / g and u = d / g (invertible mod L),
// the walk stays in the coset r = s_j mod g and equals T_r(t_j + k) for
//     T_r(t) = row((r + d t) mod n),  t_j = ((s_j - r) / g) u^{-1} mod L,
// so a table of g rows of L + n entries lets every read sit at an immediate
// offset k from the lane's own start, with no address arithmetic in the
// loop.  A stride d = 0 (an axis direction) reads one entry per lane.  The
// job weight cw = W_j / n^4 is folded in, split evenly between the real and
// imaginary parts of the transform (sgn(cw) sqrt|cw| on the line row,
// sqrt|cw| on the plane row), so the gain is accumulated as acc += g h.
// n is a power of two here.
struct JtWalk {
    int d, g, L, uinv, size;
};

template <int N>
__device__ __forceinline__ JtWalk jt_walk(int stride)
{
    JtWalk w;
    w.d = modc<N>(stride);
    if (w.d == 0) {
        w.g = N; w.L = 1; w.uinv = 0; w.size = N;
        return w;
    }
    w.g = w.d & -w.d;
    w.L = N / w.g;
    const uint32_t u = (uint32_t)(w.d / w.g);
    uint32_t x = u;   // Newton steps (mod 2^32) for the inverse of an odd u modulo a power of two
    x *= 2u - u * x;
    x *= 2u - u * x;
    x *= 2u - u * x;
    w.uinv = (int)(x & (uint32_t)(w.L - 1));
    w.size = w.g * (w.L + N);
    return w;
}

// Table entry i of a walk: row index (r + d t) mod n with r = i / (L + n), t = i mod (L + n).
template <int N>
__device__ __forceinline__ int jt_row_index(const JtWalk& w, int i)
{
    if (w.d == 0) return i;
    const int r = i / (w.L + N), t = i - r * (w.L + N);
    return (r + w.d * t) & (N - 1);
}

// Lane start inside a walk's table.
template <int N>
__device__ __forceinline__ int jt_lane_start(const JtWalk& w, int s)
{
    if (w.d == 0) return s;
    const int r = s & (w.g - 1);
    const int t = ((s / w.g) * w.uinv) & (w.L - 1);
    return r * (w.L + N) + t;
}

template <int N>
__device__ __forceinline__ void build_job_table(float* jtab, const DevPlan& pl, const float* __restrict__ jobw,
                                                int tid, int nthreads)
{
    const int arow0 = (pl.ntilde + 1) * N;
    int off = 0;
    for (int jb = 0; jb < pl.njobs; ++jb) {
        const JobDesc J = gload(pl.jobs, jb);
        const float cw = gload(jobw, jb);
        const float sq = __builtin_sqrtf(__builtin_fabsf(cw));
        const JtWalk wa = jt_walk<N>(J.e[1]), wb = jt_walk<N>(J.e[0]);
        const float* arow = pl.dirichlet + arow0 + J.M * N;
        const float* drow = pl.dirichlet + J.M * N;
        const float sa = cw < 0.f ? -sq : sq;
        for (int i = tid; i < wa.size; i += nthreads) jtab[off + i] = sa * gload(arow, jt_row_index<N>(wa, i));
        off += wa.size;
        for (int i = tid; i < wb.size; i += nthreads) jtab[off + i] = sq * gload(drow, jt_row_index<N>(wb, i));
        off += wb.size;
    }
}

// One job's spectral multiply from its tables: z(k) = (a + i b)(k) fhat(k);
// BC: the walk of b has stride 0 (one entry for the lane).
// Elements k and n - k are formed together: the lane reads its own half row
// (k <= n/2) of the spectrum, and element n - k, the conjugate of the mirror
// row's element k, comes by shuffle from the mirror lane (mlane), which has
// just read it; the tables hold entry n - k at offset n - k.
template <int N, bool BC>
__device__ __forceinline__ void jt_multiply(float2 (&z)[N], const HalfSpec<N, N * 8>& hs, const float* pa,
                                            const float* pb, int mlane)
{
    const lds_fptr la = (lds_fptr)pa;
    const lds_fptr lb = (lds_fptr)pb;
    float b0 = 0.f;
    if constexpr (BC) b0 = lb[0];
    // every spectrum load of the half row in flight at once: the transform's
    // registers are free here, and one wait per job replaces one per chunk
    // (chunks of 8 left the headline 4 % slower)
    constexpr int C = N / 2 + 1;
#pragma unroll
    for (int k0 = 0; k0 <= N / 2; k0 += C) {
        float2 F[C];
#pragma unroll
        for (int i = 0; i < C; ++i)
            if (k0 + i <= N / 2) F[i] = hs.get(k0 + i);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const int k = k0 + i;
            if (k > N / 2) break;
            const float al = la[k], ap = BC ? b0 : lb[k];
            z[k] = make_float2(__builtin_fmaf(al, F[i].x, -ap * F[i].y), __builtin_fmaf(al, F[i].y, ap * F[i].x));
            if (k >= 1 && k < N / 2) {
                const float2 Fm = make_float2(__shfl(F[i].x, mlane, 64), -__shfl(F[i].y, mlane, 64));
                const float bl = la[N - k], bp = BC ? b0 : lb[N - k];
                z[N - k] = make_float2(__builtin_fmaf(bl, Fm.x, -bp * Fm.y), __builtin_fmaf(bl, Fm.y, bp * Fm.x));
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// JT: the job loop reads the per-job tables (build_job_table) from jtab instead
// of the shared Dirichlet rows of dtab (which it then does not touch).
template <int N, int RV, bool JT = false>
__device__ __forceinline__ void cell2d_eval(const DevPlan& pl, const Item2D& it, rsrc_t rlam,
                                            const float* __restrict__ jobw, float dt, bool valid, float* xb,
                                            const float* dtab, int j, rsrc_t rsc, bool flush,
                                            const float* jtab = nullptr)
{
    constexpr int RS = N * 4;   // element stride in bytes
    float2 z[N];
#pragma unroll
    for (int i = 0; i < N; ++i) z[i] = make_float2(bload(it.f, it.vcell, i * RS), 0.f);
    fwd2d<N, RV>(z, xb, j);
    const HalfSpec<N, N * 8> fh = half2d<N>(it.fh, it.vspec, j);
    fh.put(z);

    // loss: l = Re IFFT(Lambda fhat); acc = -f l
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const float l = bload(rlam, j * 4, k * RS);
        z[k].x *= l;
        z[k].y *= l;
    }
    inv2d<N, RV>(z, xb, j);
    float acc[N];
    {
        const int vc = reread(it.vcell);
        constexpr int C = N < 16 ? N : 16;
#pragma unroll
        for (int i0 = 0; i0 < N; i0 += C) {
            float fv[C];
            load_run<C>(fv, it.f, vc, i0, RS);
#pragma unroll
            for (int i = 0; i < C; ++i) acc[i0 + i] = -fv[i] * z[i0 + i].x;
        }
    }

    // direction loop: g + i h = IFFT((alpha + i alpha') fhat), acc += W g h
    const float* atab = dtab_alpha(dtab, pl);
    int jt_off = 0;
    for (int jb = 0; jb < pl.njobs; ++jb) {
        const JobDesc J = gload(pl.jobs, jb);
        if constexpr (JT) {
            const JtWalk wa = jt_walk<N>(J.e[1]), wb = jt_walk<N>(J.e[0]);
            const float* pa = jtab + jt_off + jt_lane_start<N>(wa, modc<N>(J.e[0] * j));
            const float* pb = jtab + jt_off + wa.size + jt_lane_start<N>(wb, modc<N>(-J.e[1] * j));
            jt_off += wa.size + wb.size;
            // an axis job has one walk of stride 0; when it is the line walk the two swap
            // roles (the transform then yields h + i g, and the gain g h is the same product)
            const int mlane = (int)(threadIdx.x & 63) - j + ((N - j) & (N - 1));
            if (wb.d == 0) jt_multiply<N, true>(z, fh, pa, pb, mlane);
            else if (wa.d == 0) jt_multiply<N, true>(z, fh, pb, pa, mlane);
            else jt_multiply<N, false>(z, fh, pa, pb, mlane);
            inv2d<N, RV>(z, xb, j);
#pragma unroll
            for (int i = 0; i < N; ++i) acc[i] = __builtin_fmaf(z[i].x, z[i].y, acc[i]);
        } else {
            const float cw = gload(jobw, jb);
            job2d_multiply<N, (N == 64 ? 64 : (N < 8 ? N : 8))>(z, fh, J, dtab, atab, j);
            inv2d<N, RV>(z, xb, j);
#pragma unroll
            for (int i = 0; i < N; ++i) acc[i] = __builtin_fmaf(cw * z[i].x, z[i].y, acc[i]);
        }
        if (flush && ((jb + 1) % kFlushJobs == 0 || jb + 1 == pl.njobs))
            flush_gain<N>(acc, rsc, it.vspec, jb < kFlushJobs);
    }
    if (flush) {
        constexpr int RS2 = N * 8, C = N < 16 ? N : 16;
#pragma unroll
        for (int i0 = 0; i0 < N; i0 += C) {
            float2 sc[C];
#pragma unroll
            for (int i = 0; i < C; ++i) sc[i] = bload2(rsc, it.vspec, (i0 + i) * RS2);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < C; ++i) acc[i0 + i] = sc[i].x - sc[i].y;
        }
    }

    if (!valid) return;
    if (dt == 0.f) {
#pragma unroll
        for (int i = 0; i < N; ++i) bstore(acc[i], it.q, it.vcell, i * RS);
    } else {
        float fv[N];
        load_run<N>(fv, it.f, reread(it.vcell), 0, RS);
#pragma unroll
        for (int i = 0; i < N; ++i) bstore(__builtin_fmaf(dt, acc[i], fv[i]), it.q, it.vcell, i * RS);
    }
}


// Bilinear operator Q(g, f) of one 2D cell: gain g(i+k) f(i+l), loss
// g(i) f(i+k+l) (Sec. 2.3 states consistency for D(g, f); its Fourier form
// of Sec. 3.1 carries g~_K f~_L).  The transforms of g and f are kept as half
// spectra in two slots (rgh, it.fh); each direction is one inverse transform
// of alpha_p ghat + i alpha'_p fhat, real part the line sum of g along e_p,
// imaginary part the plane sum of f.  A job of the plan that pairs e with
// e_perp runs two transforms here: the shared transform of Q(f, f) rests on
// its symmetry under exchanging the two lines (Remark 3.5), which Q(g, f)
// lacks.  rlam: Lambda = sum_p w_p alpha_p alpha'_p over the unpaired
// directions (/ n^2); dirw: per-direction weights / n^4.  it.f holds f, rg
// holds g; the Euler form updates g: q = g + dt Q(g, f).
template <int N, int RV>
__device__ __forceinline__ void cell2d_eval_bilinear(const DevPlan& pl, const Item2D& it, rsrc_t rg, rsrc_t rgh,
                                                     rsrc_t rlam, const float* __restrict__ dirw, float dt,
                                                     bool valid, float* xb, const float* dtab, int j)
{
    constexpr int RS = N * 4;
    float2 z[N];
#pragma unroll
    for (int i = 0; i < N; ++i) z[i] = make_float2(bload(rg, it.vcell, i * RS), 0.f);
    fwd2d<N, RV>(z, xb, j);
    const HalfSpec<N, N * 8> gh = half2d<N>(rgh, it.vspec, j);
    gh.put(z);
#pragma unroll
    for (int i = 0; i < N; ++i) z[i] = make_float2(bload(it.f, it.vcell, i * RS), 0.f);
    fwd2d<N, RV>(z, xb, j);
    const HalfSpec<N, N * 8> fh = half2d<N>(it.fh, it.vspec, j);
    fh.put(z);

    // loss: l = Re IFFT(Lambda fhat); acc = -g l
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const float l = bload(rlam, j * 4, k * RS);
        z[k].x *= l;
        z[k].y *= l;
    }
    inv2d<N, RV>(z, xb, j);
    float acc[N];
    {
        const int vc = reread(it.vcell);
        constexpr int C = N < 16 ? N : 16;
#pragma unroll
        for (int i0 = 0; i0 < N; i0 += C) {
            float gv[C];
            load_run<C>(gv, rg, vc, i0, RS);
#pragma unroll
            for (int i = 0; i < C; ++i) acc[i0 + i] = -gv[i] * z[i0 + i].x;
        }
    }

    // directions: u + i v = IFFT(alpha ghat + i alpha' fhat), acc += w u v
    const float* atab = dtab_alpha(dtab, pl);
    for (int jb = 0; jb < pl.njobs; ++jb) {
        const JobDesc J = gload(pl.jobs, jb);
        const int nt = J.pp >= 0 ? 2 : 1;
        for (int t = 0; t < nt; ++t) {
            // t = 0: line e (alpha = D_M(e.K) - 1), plane e_perp (alpha' = D_M(e_perp.K));
            // t = 1: the perpendicular direction, the two roles exchanged.  Along the lane's
            // row K0 = j, e.K starts at e_0 j and steps by e_1; e_perp.K at -e_1 j, step e_0.
            const float cw = gload(dirw, t ? J.pp : J.p);
            const int se = modc<N>(J.e[0] * j), de = modc<N>(J.e[1]);
            const int sp = modc<N>(-J.e[1] * j), dp = modc<N>(J.e[0]);
            RowWalk<N> a(atab + J.M * N, t ? sp : se, t ? dp : de);
            RowWalk<N> b(dtab + J.M * N, t ? se : sp, t ? de : dp);
            if constexpr (N == 64) {
                // elements k and n - k together: the lane reads its own half rows of
                // both spectra; element n - k, the conjugate of the mirror row's
                // element k, comes by shuffle from the mirror lane (backward walks)
                const int mlane = (int)(threadIdx.x & 63) - j + ((N - j) & (N - 1));
                RowWalk<N> am(atab + J.M * N, modc<N>((t ? sp : se) - (t ? dp : de)), modc<N>(-(t ? dp : de)));
                RowWalk<N> bm(dtab + J.M * N, modc<N>((t ? se : sp) - (t ? de : dp)), modc<N>(-(t ? de : dp)));
                constexpr int H = N / 2 + 1, CH = H;   // every read of both half rows in flight at once
#pragma unroll
                for (int k0 = 0; k0 < H; k0 += CH) {
                    float2 G[CH], F[CH];
#pragma unroll
                    for (int i = 0; i < CH; ++i)
                        if (k0 + i < H) {
                            G[i] = gh.get(k0 + i);
                            F[i] = fh.get(k0 + i);
                        }
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int i = 0; i < CH; ++i) {
                        const int k = k0 + i;
                        if (k >= H) break;
                        const float al = a.get(), ap = b.get();
                        z[k] = make_float2(__builtin_fmaf(al, G[i].x, -ap * F[i].y),
                                           __builtin_fmaf(al, G[i].y, ap * F[i].x));
                        a.next();
                        b.next();
                        if (k >= 1 && k < N / 2) {
                            const float2 Gm = make_float2(__shfl(G[i].x, mlane, 64), -__shfl(G[i].y, mlane, 64));
                            const float2 Fm = make_float2(__shfl(F[i].x, mlane, 64), -__shfl(F[i].y, mlane, 64));
                            const float bl = am.get(), bp = bm.get();
                            z[N - k] = make_float2(__builtin_fmaf(bl, Gm.x, -bp * Fm.y),
                                                   __builtin_fmaf(bl, Gm.y, bp * Fm.x));
                            am.next();
                            bm.next();
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
                inv2d<N, RV>(z, xb, j);
#pragma unroll
                for (int i = 0; i < N; ++i) acc[i] = __builtin_fmaf(cw * z[i].x, z[i].y, acc[i]);
                continue;
            }
            // chunks of 8 elements of both spectra, all read before the chunk's
            // multiply (at n = 64 chunks of 2 left most of each read's latency
            // exposed: 2.53 against 1.96 ms for 16384 cells at P = 16)
            constexpr int C = N < 8 ? N : 8;
#pragma unroll
            for (int k0 = 0; k0 < N; k0 += C) {
                float2 G[C], F[C];
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    G[i] = gh.get(k0 + i);
                    F[i] = fh.get(k0 + i);
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    const float al = a.get(), ap = b.get();
                    z[k0 + i] = make_float2(__builtin_fmaf(al, G[i].x, -ap * F[i].y),
                                            __builtin_fmaf(al, G[i].y, ap * F[i].x));
                    a.next();
                    b.next();
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            inv2d<N, RV>(z, xb, j);
#pragma unroll
            for (int i = 0; i < N; ++i) acc[i] = __builtin_fmaf(cw * z[i].x, z[i].y, acc[i]);
        }
    }

    if (!valid) return;
    if (dt == 0.f) {
#pragma unroll
        for (int i = 0; i < N; ++i) bstore(acc[i], it.q, it.vcell, i * RS);
    } else {
        float gv[N];
        load_run<N>(gv, rg, reread(it.vcell), 0, RS);
#pragma unroll
        for (int i = 0; i < N; ++i) bstore(__builtin_fmaf(dt, acc[i], gv[i]), it.q, it.vcell, i * RS);
    }
}


// Sum of a double over the n lanes of an aligned lane group.
template <int N>
__device__ __forceinline__ double group_sumd(double v)
{
#pragma unroll
    for (int o = N / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Near-equilibrium evaluation of one 2D cell.  With M the Maxwellian of the
// cell's moments (FP64) and g = f - M, the bilinear identity
//     Q(f, f) - Q(M, M) = Q(g, f) + Q(M, g)
// is evaluated with every transform carrying either f-sized or g-sized data,
// never both (a small signal packed with a large one in one complex transform
// inherits rounding of the large one's size):
//     gain_j = line_j(g) plane_j(f) + (line_j(f) - line_j(g)) plane_j(g)
//     loss   = g l(f) + M l(g).
// Q(M, M) vanishes except for aliasing (every bracket of an unwrapped discrete
// Maxwellian cancels in the pair sum of Sec. 2.3), and is left out: the result is
// Q(f, f) - Q(M, M).  Errors scale with |f| |g| instead of |f|^2.
// M is recomputed from its parameters where needed (FP64 exp) instead of being
// kept in registers.  With STAGE the transform of g of each job is parked in
// the buffer rtg (same layout as the spectra) while the transform of f is
// formed, for launches whose register budget cannot hold both.
template <int N, int RV, bool STAGE>
__device__ __forceinline__ void cell2d_eval_split(const DevPlan& pl, const Item2D& it, rsrc_t rgh, rsrc_t rtg,
                                                  rsrc_t rlam, const float* __restrict__ jobw, float dt, bool valid,
                                                  float* xb, const float* dtab, int j)
{
    constexpr int RS = N * 4, RS2 = N * 8;
    // moments in index units (column j holds the points (i, j)), FP64
    constexpr int C = N < 16 ? N : 16;   // elements per read chunk
    double s0 = 0.0, sa = 0.0, s2 = 0.0;
#pragma unroll
    for (int i0 = 0; i0 < N; i0 += C) {
        float fv[C];
        load_run<C>(fv, it.f, it.vcell, i0, RS);
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const double v = fv[i];
            s0 += v;
            sa += (double)(i0 + i) * v;
            s2 += (double)((i0 + i) * (i0 + i)) * v;
        }
    }
    double sb = (double)j * s0;
    s2 += (double)(j * j) * s0;
    s0 = group_sumd<N>(s0);
    sa = group_sumd<N>(sa);
    sb = group_sumd<N>(sb);
    s2 = group_sumd<N>(s2);
    const double m0 = sa / s0, m1 = sb / s0;
    const double var = 0.5 * (s2 / s0 - m0 * m0 - m1 * m1);
    // a cell without a usable Gaussian fit keeps M = 0, i.e. the plain evaluation
    // (its parameters are replaced so that no NaN of 0/0 reaches M)
    const bool ok = s0 > 0.0 && var > 0.25 && __builtin_isfinite(var) && __builtin_isfinite(m0) &&
                    __builtin_isfinite(m1);
    const double mu0 = ok ? m0 : 0.0, mu1 = ok ? m1 : 0.0;
    const double inv2v = ok ? 0.5 / var : 0.0;
    const double ej = ok ? s0 / (2.0 * kPi * var) * exp(-(j - mu1) * (j - mu1) * inv2v) : 0.0;
    // M(i, j) in FP64
#define QDVM_MAXW(i) (ej * exp(-((i) - mu0) * ((i) - mu0) * inv2v))

    float2 z[N];
#pragma unroll
    for (int i0 = 0; i0 < N; i0 += C) {
        float fv[C];
        load_run<C>(fv, it.f, it.vcell, i0, RS);
#pragma unroll
        for (int i = 0; i < C; ++i) z[i0 + i] = make_float2((float)((double)fv[i] - QDVM_MAXW(i0 + i)), 0.f);
    }
    fwd2d<N, RV>(z, xb, j);
    const HalfSpec<N, N * 8> gh = half2d<N>(rgh, it.vspec, j), fh = half2d<N>(it.fh, it.vspec, j);
    gh.put(z);
#pragma unroll
    for (int k0 = 0; k0 < N; k0 += C) {
        float l[C];
        load_run<C>(l, rlam, j * 4, k0, RS);
#pragma unroll
        for (int k = 0; k < C; ++k) {
            z[k0 + k].x *= l[k];
            z[k0 + k].y *= l[k];
        }
    }
    inv2d<N, RV>(z, xb, j);                      // l(g)
    float acc[N];                                // holds l(g) until l(f) is formed
#pragma unroll
    for (int i = 0; i < N; ++i) acc[i] = z[i].x;
    {
        const int vc = reread(it.vcell);
#pragma unroll
        for (int i = 0; i < N; ++i) z[i] = make_float2(bload(it.f, vc, i * RS), 0.f);
    }
    fwd2d<N, RV>(z, xb, j);
    fh.put(z);
#pragma unroll
    for (int k0 = 0; k0 < N; k0 += C) {
        float l[C];
        load_run<C>(l, rlam, j * 4, k0, RS);
#pragma unroll
        for (int k = 0; k < C; ++k) {
            z[k0 + k].x *= l[k];
            z[k0 + k].y *= l[k];
        }
    }
    inv2d<N, RV>(z, xb, j);                      // l(f)
    {
        // M again (kept opaque so it is not carried over from the first evaluation)
        const double iv = opaque(inv2v), m0 = opaque(mu0);
        const int vc = reread(it.vcell);
#pragma unroll
        for (int i0 = 0; i0 < N; i0 += C) {
            float fv[C];
            load_run<C>(fv, it.f, vc, i0, RS);
#pragma unroll
            for (int i = 0; i < C; ++i) {
                const double m = ej * exp(-((i0 + i) - m0) * ((i0 + i) - m0) * iv);
                const float g = (float)((double)fv[i] - m);
                acc[i0 + i] = -__builtin_fmaf(g, z[i0 + i].x, (float)m * acc[i0 + i]);
            }
        }
    }
#undef QDVM_MAXW

    const float* atab = dtab_alpha(dtab, pl);
    for (int jb = 0; jb < pl.njobs; ++jb) {
        const JobDesc J = gload(pl.jobs, jb);
        const float cw = gload(jobw, jb);
        float2 tg[N];
        job2d_multiply<N>(tg, gh, J, dtab, atab, j);
        inv2d<N, RV>(tg, xb, j);                 // line(g) + i plane(g)
        if constexpr (STAGE) {
#pragma unroll
            for (int i = 0; i < N; ++i) bstore2(tg[i], rtg, it.vspec, i * RS2);
        }
        job2d_multiply<N>(z, fh, J, dtab, atab, j);
        inv2d<N, RV>(z, xb, j);                  // line(f) + i plane(f)
        if constexpr (STAGE) {
            // the parked transform of g, read a chunk at a time before use
#pragma unroll
            for (int i0 = 0; i0 < N; i0 += 8) {
                float2 t[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) t[i] = bload2(rtg, it.vspec, (i0 + i) * RS2);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const float gain = __builtin_fmaf(t[i].x, z[i0 + i].y, (z[i0 + i].x - t[i].x) * t[i].y);
                    acc[i0 + i] = __builtin_fmaf(cw, gain, acc[i0 + i]);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const float gain = __builtin_fmaf(tg[i].x, z[i].y, (z[i].x - tg[i].x) * tg[i].y);
                acc[i] = __builtin_fmaf(cw, gain, acc[i]);
            }
        }
    }

    if (!valid) return;
    if (dt == 0.f) {
#pragma unroll
        for (int i = 0; i < N; ++i) bstore(acc[i], it.q, it.vcell, i * RS);
    } else {
        float fv[N];
        load_run<N>(fv, it.f, reread(it.vcell), 0, RS);
#pragma unroll
        for (int i = 0; i < N; ++i) bstore(__builtin_fmaf(dt, acc[i], fv[i]), it.q, it.vcell, i * RS);
    }
}

// A double that is the same in every lane of the wave, moved to scalar registers.
__device__ __forceinline__ double uniform(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// The near-equilibrium evaluation with two waves per cell, for n = 64, where
// one pencil fills half of a lane's registers: a wave that held both transforms
// of a job and the accumulator ran at one wave per SIMD.  Here the g wave forms
// every transform of g = f - M and the f wave every transform of f, each in its
// own LDS slot (xg, xf).  A job's gain is split between the two accumulators,
//     line(g) (plane(f) - plane(g))    in the g wave,
//     line(f) plane(g)                 in the f wave,
// (together line(g) plane(f) + line(M) plane(g), each term of size |f| |g|),
// so that each wave hands the other only its plane field, through its own
// slot.  The f wave's accumulator joins the g wave's at the end, which writes
// the result.  All waves of the workgroup run the same number of cells.
template <int N, int RV>
__device__ __forceinline__ void cell2d_eval_split_pair(const DevPlan& pl, const Item2D& it, rsrc_t rgh,
                                                       rsrc_t rlam, const float* __restrict__ jobw, float dt,
                                                       bool valid, float* xg, float* xf, const float* dtab, int j,
                                                       bool fwave)
{
    static_assert(N == 64, "one cell per wave: lane j holds column j");
    constexpr int RS = N * 4;
    float* own = fwave ? xf : xg;
    const float* other = fwave ? xg : xf;
    // the previous cell's last hand-over has been read from both slots
    __syncthreads();
    double ej = 0.0, mu0 = 0.0, inv2v = 0.0;
    float2 z[N];
    if (fwave) {
#pragma unroll
        for (int i = 0; i < N; ++i) z[i] = make_float2(bload(it.f, it.vcell, i * RS), 0.f);
    } else {
        // moments in index units (column j holds the points (i, j)), FP64
        double s0 = 0.0, sa = 0.0, s2 = 0.0;
#pragma unroll
        for (int i0 = 0; i0 < N; i0 += 16) {
            float fv[16];
            load_run<16>(fv, it.f, it.vcell, i0, RS);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const double v = fv[i];
                s0 += v;
                sa += (double)(i0 + i) * v;
                s2 += (double)((i0 + i) * (i0 + i)) * v;
            }
        }
        double sb = (double)j * s0;
        s2 += (double)(j * j) * s0;
        s0 = group_sumd<N>(s0);
        sa = group_sumd<N>(sa);
        sb = group_sumd<N>(sb);
        s2 = group_sumd<N>(s2);
        const double m0 = sa / s0, m1 = sb / s0;
        const double var = 0.5 * (s2 / s0 - m0 * m0 - m1 * m1);
        const bool ok = s0 > 0.0 && var > 0.25 && __builtin_isfinite(var) && __builtin_isfinite(m0) &&
                        __builtin_isfinite(m1);
        // the moments are sums over the whole wave: uniform, kept in scalar registers
        mu0 = uniform(ok ? m0 : 0.0);
        const double mu1 = ok ? m1 : 0.0;
        inv2v = uniform(ok ? 0.5 / var : 0.0);
        ej = ok ? s0 / (2.0 * kPi * var) * exp(-(j - mu1) * (j - mu1) * inv2v) : 0.0;
        // M(i, j) = ej e_i: the n factors e_i are the same in every lane; lane
        // j forms e_j, in the wave's own slot (free until its transform)
        double* ex = reinterpret_cast<double*>(xg);
        ex[j] = exp(-(j - mu0) * (j - mu0) * inv2v);
        wave_sync();
        const int vc = reread(it.vcell);
#pragma unroll
        for (int i0 = 0; i0 < N; i0 += 16) {
            float fv[16];
            double e[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) e[i] = ex[i0 + i];
            load_run<16>(fv, it.f, vc, i0, RS);
#pragma unroll
            for (int i = 0; i < 16; ++i) z[i0 + i] = make_float2((float)((double)fv[i] - ej * e[i]), 0.f);
        }
    }
    fwd2d<N, RV>(z, own, j);
    const HalfSpec<N, N * 8> sp = half2d<N>(fwave ? it.fh : rgh, it.vspec, j);
    sp.put(z);
#pragma unroll
    for (int k0 = 0; k0 < N; k0 += 16) {
        float l[16];
        load_run<16>(l, rlam, j * 4, k0, RS);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            z[k0 + k].x *= l[k];
            z[k0 + k].y *= l[k];
        }
    }
    inv2d<N, RV>(z, own, j);                     // l(g) or l(f)
    // loss g l(f) + M l(g): the f wave hands l(f) over (its slot is free once
    // every lane of the wave has read its transpose)
    if (fwave) {
        wave_sync();
#pragma unroll
        for (int i = 0; i < N; ++i) xf[i * N + j] = z[i].x;
    }
    __syncthreads();
    float acc[N];
    if (fwave) {
#pragma unroll
        for (int i = 0; i < N; ++i) acc[i] = 0.f;
    } else {
        // the factors e_i again, in the own slot (free after the transform)
        double* ex = reinterpret_cast<double*>(xg);
        wave_sync();
        ex[j] = exp(-(j - mu0) * (j - mu0) * inv2v);
        wave_sync();
        const int vc = reread(it.vcell);
#pragma unroll
        for (int i0 = 0; i0 < N; i0 += 16) {
            float fv[16], lf[16];
            double e[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                e[i] = ex[i0 + i];
                lf[i] = xf[(i0 + i) * N + j];
            }
            load_run<16>(fv, it.f, vc, i0, RS);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const double m = ej * e[i];
                const float g = (float)((double)fv[i] - m);
                acc[i0 + i] = -__builtin_fmaf(g, lf[i], (float)m * z[i0 + i].x);
            }
        }
    }

    // per job: line + i plane of this wave's function, then the other wave's plane
    const float sub = fwave ? 0.f : 1.f;
    const float* atab = dtab_alpha(dtab, pl);
    for (int jb = 0; jb < pl.njobs; ++jb) {
        const JobDesc J = gload(pl.jobs, jb);
        const float cw = gload(jobw, jb);
        job2d_multiply<N, 64>(z, sp, J, dtab, atab, j);   // the whole row's reads in flight at once
        __syncthreads();                         // the other wave has read this slot
        inv2d<N, RV>(z, own, j);
        wave_sync();
#pragma unroll
        for (int i = 0; i < N; ++i) own[i * N + j] = z[i].y;
        __syncthreads();
        // the other wave's plane, read a chunk at a time before use
#pragma unroll
        for (int i0 = 0; i0 < N; i0 += 16) {
            float o[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) o[i] = other[(i0 + i) * N + j];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const float t = __builtin_fmaf(-sub, z[i0 + i].y, o[i]);
                acc[i0 + i] = __builtin_fmaf(cw * z[i0 + i].x, t, acc[i0 + i]);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    __syncthreads();                             // both planes of the last job have been read
    if (fwave) {
#pragma unroll
        for (int i = 0; i < N; ++i) xf[i * N + j] = acc[i];
    }
    __syncthreads();
    if (fwave || !valid) return;
#pragma unroll
    for (int i0 = 0; i0 < N; i0 += 16) {
        float a2[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) a2[i] = xf[(i0 + i) * N + j];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i0 + i] += a2[i];
    }
    if (dt == 0.f) {
#pragma unroll
        for (int i = 0; i < N; ++i) bstore(acc[i], it.q, it.vcell, i * RS);
    } else {
        float fv[N];
        load_run<N>(fv, it.f, reread(it.vcell), 0, RS);
#pragma unroll
        for (int i = 0; i < N; ++i) bstore(__builtin_fmaf(dt, acc[i], fv[i]), it.q, it.vcell, i * RS);
    }
}

// Adjoint of one 2D cell; the algebra is written out above cell3d_vjp (R, the
// Hermitian accumulator S).  The mirror row -K0 of the lane's row K0 = j is
// another lane of the same wave: uhat(-K) comes by shuffle.  rr: the table R
// (half rows, 4 bytes per element) in the second spectral slot; rnone: a
// descriptor of the accumulator's base with extent 0.
template <int N, int RV>
__device__ __forceinline__ void cell2d_vjp(const DevPlan& pl, const Item2D& it, rsrc_t rc, rsrc_t rr,
                                           rsrc_t rsh, rsrc_t rnone, rsrc_t rlam, const float* __restrict__ jobw,
                                           double* __restrict__ gwp, bool gw_first, bool valid, float inv_n2,
                                           float inv_n, float* xb, const float* dtab, int j)
{
    constexpr int RS = N * 4, RS2 = N * 8;
    const int mrow = (N - j) & (N - 1);                          // mirror row
    const int mlane = (int)(threadIdx.x & 63) - j + mrow;        // its lane in the wave
    const int rown = it.vspec / 2;                               // R: own row offset
    float2 z[N];
#pragma unroll
    for (int i = 0; i < N; ++i) z[i] = make_float2(bload(it.f, it.vcell, i * RS), 0.f);
    fwd2d<N, RV>(z, xb, j);
    const HalfSpec<N, N * 8> fh = half2d<N>(it.fh, it.vspec, j);
    fh.put(z);
#pragma unroll
    for (int i = 0; i < N; ++i)
        z[i] = make_float2(bload(rc, it.vcell, i * RS) * bload(it.f, it.vcell, i * RS), 0.f);
    fwd2d<N, RV>(z, xb, j);
    // R = Re(conj F(cf) fhat) on the own half row (written by this lane); the
    // reads of a chunk are issued before its stores, which the compiler cannot
    // tell apart from them
    constexpr int CR = N / 2 + 1 < 17 ? N / 2 + 1 : 17;
#pragma unroll
    for (int k0 = 0; k0 <= N / 2; k0 += CR) {
        constexpr int C = CR;
        float2 F[C];
#pragma unroll
        for (int i = 0; i < C; ++i)
            if (k0 + i <= N / 2) F[i] = fh.get(k0 + i);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < C; ++i)
            if (k0 + i <= N / 2)
                bstore(__builtin_fmaf(z[k0 + i].x, F[i].x, z[k0 + i].y * F[i].y), rr, rown, (k0 + i) * RS);
    }
    // IFFT(Lambda (fhat + i F(cf))) = l + i C_Lambda(cf)
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const float2 F = fh.get(k);
        const float l = bload(rlam, j * 4, k * RS);
        z[k] = make_float2(l * (F.x - z[k].y), l * (F.y + z[k].x));
        QDVM_CHUNK_FENCE(k);
    }
    inv2d<N, RV>(z, xb, j);
    // -c l - C(cf) goes to grad_f now and is completed after the direction
    // loop, so that no pencil-sized accumulator stays live through it
    {
        float cv[N];
        load_run<N>(cv, rc, it.vcell, 0, RS);
#pragma unroll
        for (int i = 0; i < N; ++i) bstore(-cv[i] * z[i].x - z[i].y, it.q, it.vcell, i * RS);
    }

    // The accumulator S lives in memory between jobs, in half rows.  The first
    // job reads it through an empty descriptor (the hardware returns 0 for every
    // read and drops every write, with no memory request), so it needs no zero
    // fill; the last job keeps its sums in z, the final transform's input, and
    // writes through the empty descriptor instead of storing them to be read
    // back.
    const float* atab = dtab_alpha(dtab, pl);
    for (int jb = 0; jb < pl.njobs; ++jb) {
        const JobDesc J = gload(pl.jobs, jb);
        const float cw = gload(jobw, jb);
        const rsrc_t rsr = jb == 0 ? rnone : rsh;
        const rsrc_t rsw = jb + 1 == pl.njobs ? rnone : rsh;
        float spart = 0.f;
        {
            // elements k and n - k together: the lane reads its own half row (k <= n/2)
            // of the spectrum and of R; element n - k is the conjugate (for R the
            // value) of the mirror row's element k, which the mirror lane has just
            // read, so it comes by shuffle instead of a second read from memory.
            // Forward walks for k, backward walks (from k = n - 1) for n - k.
            RowWalk<N> a(atab + J.M * N, modc<N>(J.e[0] * j), modc<N>(J.e[1]));
            RowWalk<N> b(dtab + J.M * N, modc<N>(-J.e[1] * j), modc<N>(J.e[0]));
            RowWalk<N> am(atab + J.M * N, modc<N>(J.e[0] * j - J.e[1]), modc<N>(-J.e[1]));
            RowWalk<N> bm(dtab + J.M * N, modc<N>(-J.e[1] * j - J.e[0]), modc<N>(-J.e[0]));
            // two chunks of reads at n = 64 (one chunk of 33 reads of F and R
            // together would not leave the registers for two waves per SIMD)
            constexpr int C = N / 2 + 1 < 17 ? N / 2 + 1 : 17;
#pragma unroll
            for (int k0 = 0; k0 <= N / 2; k0 += C) {
                float2 F[C];
                float R[C];
#pragma unroll
                for (int i = 0; i < C; ++i)
                    if (k0 + i <= N / 2) {
                        F[i] = bload2(it.fh, it.vspec, (k0 + i) * RS2);
                        R[i] = bload(rr, rown, (k0 + i) * RS);
                    }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    const int k = k0 + i;
                    if (k > N / 2) break;
                    const float al = a.get(), ap = b.get();
                    z[k] = make_float2(__builtin_fmaf(al, F[i].x, -ap * F[i].y),
                                       __builtin_fmaf(al, F[i].y, ap * F[i].x));
                    spart = __builtin_fmaf(al * ap, R[i], spart);
                    a.next();
                    b.next();
                    if (k >= 1 && k < N / 2) {
                        const float2 Fm = make_float2(__shfl(F[i].x, mlane, 64), -__shfl(F[i].y, mlane, 64));
                        const float Rm = __shfl(R[i], mlane, 64);
                        const float bl = am.get(), bp = bm.get();
                        z[N - k] = make_float2(__builtin_fmaf(bl, Fm.x, -bp * Fm.y),
                                               __builtin_fmaf(bl, Fm.y, bp * Fm.x));
                        spart = __builtin_fmaf(bl * bp, Rm, spart);
                        am.next();
                        bm.next();
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        inv2d<N, RV>(z, xb, j);   // z = u + i v = n^2 (g + i h)
        float rpart = 0.f;
        {
            const int vc = reread(it.vcell);
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const float c = bload(rc, vc, i * RS);
                rpart = __builtin_fmaf(c * z[i].x, z[i].y, rpart);
                z[i] = make_float2(c * z[i].y, c * z[i].x);   // c v + i c u
                // the cotangent's reads in flight 32 at a time (1.84 -> 1.80 ms
                // at n = 64 against chunks of 8)
                if ((i & 31) == 31) __builtin_amdgcn_sched_barrier(0);
            }
        }
        // FP64 across the cell's lanes: the per-lane terms largely cancel
        const double tot = group_sumd<N>((double)rpart * inv_n2 - (double)spart * inv_n);
        if (j == 0 && valid) gw_accumulate(gwp + jb, tot, gw_first);
        fwd2d<N, RV>(z, xb, j);
        {
            // the multipliers are read again rather than kept from the first
            // multiply (holding them through two transforms costs registers)
            const int jj = reread(j);
            RowWalk<N> a(atab + J.M * N, modc<N>(J.e[0] * jj), modc<N>(J.e[1]));
            RowWalk<N> b(dtab + J.M * N, modc<N>(-J.e[1] * jj), modc<N>(J.e[0]));
            constexpr int CS = N / 2 + 1 < 8 ? N / 2 + 1 : 8;
#pragma unroll
            for (int k0 = 0; k0 <= N / 2; k0 += CS) {
                // the chunk's accumulator reads go out before its stores (the
                // compiler would otherwise wait for each read in turn)
                constexpr int C = CS;
                float2 sv[C], m[C], w[C];
#pragma unroll
                for (int i = 0; i < C; ++i)
                    if (k0 + i <= N / 2) {
                        sv[i] = bload2(rsr, it.vspec, (k0 + i) * RS2);
                        w[i] = make_float2(a.get(), b.get());
                        a.next();
                        b.next();
                    }
                // Hermitian part of (alpha - i alpha') uhat: uhat(-K) is element
                // n - k of the mirror row, another lane's
#pragma unroll
                for (int i = 0; i < C; ++i)
                    if (k0 + i <= N / 2) {
                        const int k = k0 + i;
                        m[i] = make_float2(__shfl(z[(N - k) % N].x, mlane, 64), __shfl(z[(N - k) % N].y, mlane, 64));
                    }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    const int k = k0 + i;
                    if (k > N / 2) break;
                    const float mx = m[i].x, my = m[i].y;
                    const float al = 0.5f * cw * w[i].x, ap = 0.5f * cw * w[i].y;
                    float2 t = make_float2(__builtin_fmaf(al, z[k].x + mx, ap * (z[k].y + my)),
                                           __builtin_fmaf(al, z[k].y - my, -ap * (z[k].x - mx)));
                    // z[k] is not read again in this job: element k is the
                    // mirror of n - k > n/2 (never formed here) except for k = 0
                    // and n/2, whose mirror reads precede this write
                    z[k] = make_float2(t.x + sv[i].x, t.y + sv[i].y);
                    bstore2(z[k], rsw, it.vspec, k * RS2);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    if (pl.njobs > 0) {
        // z[0..n/2] holds the own half row of S; element k > n/2 is the conjugate
        // of element n - k of the mirror row
#pragma unroll
        for (int k = N / 2 + 1; k < N; ++k)
            z[k] = make_float2(__shfl(z[N - k].x, mlane, 64), -__shfl(z[N - k].y, mlane, 64));
        inv2d<N, RV>(z, xb, j);
        {
            float gv[N];
            load_run<N>(gv, it.q, it.vcell, 0, RS);
#pragma unroll
            for (int i = 0; i < N; ++i) bstore(gv[i] + z[i].x, it.q, it.vcell, i * RS);
        }
    }
}

}  // namespace qdvm
