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
template <int N>
__device__ __forceinline__ void job2d_multiply(float2 (&z)[N], const HalfSpec<N, N * 8>& hs, const JobDesc& J,
                                               const float* dtab, const float* atab, int j)
{
    RowWalk<N> a(atab + J.M * N, modc<N>(J.e[0] * j), modc<N>(J.e[1]));
    RowWalk<N> b(dtab + J.M * N, modc<N>(-J.e[1] * j), modc<N>(J.e[0]));
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const float2 F = hs.get(k);
        const float al = a.get(), ap = b.get();
        z[k] = make_float2(__builtin_fmaf(al, F.x, -ap * F.y), __builtin_fmaf(al, F.y, ap * F.x));
        a.next();
        b.next();
        QDVM_CHUNK_FENCE(k);
    }
}

template <int N, int RV>
__device__ __forceinline__ void cell2d_eval(const DevPlan& pl, const Item2D& it, rsrc_t rlam,
                                            const float* __restrict__ jobw, float dt, bool valid, float* xb,
                                            const float* dtab, int j)
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
    for (int jb = 0; jb < pl.njobs; ++jb) {
        const JobDesc J = gload(pl.jobs, jb);
        const float cw = gload(jobw, jb);
        job2d_multiply<N>(z, fh, J, dtab, atab, j);
        inv2d<N, RV>(z, xb, j);
#pragma unroll
        for (int i = 0; i < N; ++i) acc[i] = __builtin_fmaf(cw * z[i].x, z[i].y, acc[i]);
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
    double s0 = 0.0, sa = 0.0, s2 = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const double v = bload(it.f, it.vcell, i * RS);
        s0 += v;
        sa += (double)i * v;
        s2 += (double)(i * i) * v;
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
    for (int i = 0; i < N; ++i) {
        z[i] = make_float2((float)((double)bload(it.f, it.vcell, i * RS) - QDVM_MAXW(i)), 0.f);
        QDVM_CHUNK_FENCE(i);
    }
    fwd2d<N, RV>(z, xb, j);
    const HalfSpec<N, N * 8> gh = half2d<N>(rgh, it.vspec, j), fh = half2d<N>(it.fh, it.vspec, j);
    gh.put(z);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const float l = bload(rlam, j * 4, k * RS);
        z[k].x *= l;
        z[k].y *= l;
        QDVM_CHUNK_FENCE(k);
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
    for (int k = 0; k < N; ++k) {
        const float l = bload(rlam, j * 4, k * RS);
        z[k].x *= l;
        z[k].y *= l;
        QDVM_CHUNK_FENCE(k);
    }
    inv2d<N, RV>(z, xb, j);                      // l(f)
    {
        // M again (kept opaque so it is not carried over from the first evaluation)
        const double iv = opaque(inv2v), m0 = opaque(mu0);
        const int vc = reread(it.vcell);
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const double m = ej * exp(-((i) - m0) * ((i) - m0) * iv);
            const float g = (float)((double)bload(it.f, vc, i * RS) - m);
            acc[i] = -__builtin_fmaf(g, z[i].x, (float)m * acc[i]);
            QDVM_CHUNK_FENCE(i);
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

// Adjoint of one 2D cell; the algebra is written out above cell3d_vjp (R, the
// Hermitian accumulator S).  The mirror row -K0 of the lane's row K0 = j is
// another lane of the same wave: uhat(-K) comes by shuffle.  rr: the table R
// (half rows, 4 bytes per element) in the second spectral slot.
template <int N, int RV>
__device__ __forceinline__ void cell2d_vjp(const DevPlan& pl, const Item2D& it, rsrc_t rc, rsrc_t rr,
                                           rsrc_t rsh, rsrc_t rlam, const float* __restrict__ jobw,
                                           float* __restrict__ gwp, bool valid, float inv_n2, float inv_n,
                                           float* xb, const float* dtab, int j)
{
    constexpr int RS = N * 4, RS2 = N * 8;
    const int mrow = (N - j) & (N - 1);                          // mirror row
    const int mlane = (int)(threadIdx.x & 63) - j + mrow;        // its lane in the wave
    const int rown = it.vspec / 2, rmir = rown + (mrow - j) * 4; // R: own and mirror row offsets
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
    // R = Re(conj F(cf) fhat) on the own half row (written by this lane)
#pragma unroll
    for (int k = 0; k <= N / 2; ++k) {
        const float2 F = fh.get(k);
        bstore(__builtin_fmaf(z[k].x, F.x, z[k].y * F.y), rr, rown, k * RS);
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

    // the accumulator starts at zero (an unconditional read-modify-write in the
    // job loop keeps that loop free of per-element branches)
#pragma unroll
    for (int k = 0; k <= N / 2; ++k) bstore2(make_float2(0.f, 0.f), rsh, it.vspec, k * RS2);
    const float* atab = dtab_alpha(dtab, pl);
    for (int jb = 0; jb < pl.njobs; ++jb) {
        const JobDesc J = gload(pl.jobs, jb);
        const float cw = gload(jobw, jb);
        float spart = 0.f;
        {
            RowWalk<N> a(atab + J.M * N, modc<N>(J.e[0] * j), modc<N>(J.e[1]));
            RowWalk<N> b(dtab + J.M * N, modc<N>(-J.e[1] * j), modc<N>(J.e[0]));
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const float2 F = fh.get(k);
                const float R = k <= N / 2 ? bload(rr, rown, k * RS) : bload(rr, rmir, (N - k) * RS);
                const float al = a.get(), ap = b.get();
                z[k] = make_float2(__builtin_fmaf(al, F.x, -ap * F.y), __builtin_fmaf(al, F.y, ap * F.x));
                spart = __builtin_fmaf(al * ap, R, spart);
                a.next();
                b.next();
                QDVM_CHUNK_FENCE(k);
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
                QDVM_CHUNK_FENCE(i);
            }
        }
        const float tot = group_sum<N>(rpart * inv_n2 - spart * inv_n);
        if (j == 0 && valid) gwp[jb] = tot;
        fwd2d<N, RV>(z, xb, j);
        {
            // the multipliers are read again rather than kept from the first
            // multiply (holding them through two transforms costs registers)
            const int jj = reread(j);
            RowWalk<N> a(atab + J.M * N, modc<N>(J.e[0] * jj), modc<N>(J.e[1]));
            RowWalk<N> b(dtab + J.M * N, modc<N>(-J.e[1] * jj), modc<N>(J.e[0]));
#pragma unroll
            for (int k = 0; k <= N / 2; ++k) {
                // Hermitian part of (alpha - i alpha') uhat: uhat(-K) is element
                // n - k of the mirror row
                const float mx = __shfl(z[(N - k) % N].x, mlane, 64), my = __shfl(z[(N - k) % N].y, mlane, 64);
                const float al = 0.5f * cw * a.get(), ap = 0.5f * cw * b.get();
                float2 t = make_float2(__builtin_fmaf(al, z[k].x + mx, ap * (z[k].y + my)),
                                       __builtin_fmaf(al, z[k].y - my, -ap * (z[k].x - mx)));
                const float2 sv = bload2(rsh, it.vspec, k * RS2);
                bstore2(make_float2(t.x + sv.x, t.y + sv.y), rsh, it.vspec, k * RS2);
                a.next();
                b.next();
                QDVM_CHUNK_FENCE(k);
            }
        }
    }
    if (pl.njobs > 0) {
        const HalfSpec<N, N * 8> sh = half2d<N>(rsh, it.vspec, j);
#pragma unroll
        for (int k = 0; k < N; ++k) z[k] = sh.get(k);
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
