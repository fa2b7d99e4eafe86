// The forward transform stage of the 2D evaluation, by itself, two ways: the
// register FFT of the collision kernels, and the DFT written as matrix
// products on the FP32 matrix cores (MFMA).  Used to measure which of the two
// the evaluation should run at small n (Sec. 3.1 gives the operator's Fourier
// form; a dense DFT is the textbook alternative to the FFT for short pencils).
#include "cells_2d.h"

namespace qdvm {

namespace {

// Register FFT: one cell = 16 lanes, lane j loads column j, transforms both
// axes (fwd2d), runs `reps` inverse-forward round trips in registers (each
// scaled back by 1/n^2), and writes row K0 = j of the spectrum as out[K1][K0].
__global__ __launch_bounds__(256) void k_stage_fft16(int batch, int reps, const float* __restrict__ f,
                                                     float2* __restrict__ out)
{
    constexpr int N = 16, CPB = 16, SLOT = N * (N + 1), NPTS = N * N;
    __shared__ float lds[CPB * SLOT];
    const int tid = threadIdx.x, j = tid & (N - 1), local = tid / N;
    float* xb = lds + local * SLOT;
    const int nitems = (batch + CPB - 1) / CPB;
    for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
        const int cell = item * CPB + local;
        const int nvalid = min(CPB, batch - item * CPB);
        const rsrc_t rf = make_rsrc(f + (size_t)item * CPB * NPTS, nvalid * NPTS * 4);
        const rsrc_t ro = make_rsrc(out + (size_t)item * CPB * NPTS, nvalid * NPTS * 8);
        const int v = (local * NPTS + j) * 4;
        float2 z[N];
#pragma unroll
        for (int i = 0; i < N; ++i) z[i] = make_float2(bload(rf, v, i * N * 4), 0.f);
        fwd2d<N, 0>(z, xb, j);
        for (int r = 0; r < reps; ++r) {
            inv2d<N, 0>(z, xb, j);
#pragma unroll
            for (int i = 0; i < N; ++i) z[i] = make_float2(z[i].x * (1.f / NPTS), z[i].y * (1.f / NPTS));
            fwd2d<N, 0>(z, xb, j);
        }
        if (cell < batch) {
#pragma unroll
            for (int k = 0; k < N; ++k) bstore2(z[k], ro, (local * NPTS + j) * 8, k * N * 8);
        }
    }
}

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Complex 16 x 16 matrices on the matrix cores, one per wave.
// v_mfma_f32_16x16x4_f32 operand layout: A[i][k] in lane i + 16 k, B[k][j] in
// lane j + 16 k, D[i][j] in lane j + 16 (i / 4), register i % 4; a product over
// K = 16 is four such steps s (k = 4 s + lane / 16).  Results move between
// products through the wave's LDS rows ([row][col], stride 17).
struct Cmat {
    floatx4 re, im;
};

// D-layout matrix -> LDS
__device__ __forceinline__ void cm_store(const Cmat& m, float* lr, float* li, int q, int c)
{
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        lr[(4 * q + r) * 17 + c] = m.re[r];
        li[(4 * q + r) * 17 + c] = m.im[r];
    }
}

// Y = Wx M, Wx = W or conj(W) (wi already negated for conj), M read from LDS as the B operand
__device__ __forceinline__ Cmat cm_w_times(const float (&wr)[4], const float (&wi)[4], const float* lr,
                                           const float* li, int q, int c)
{
    floatx4 yr = {0.f, 0.f, 0.f, 0.f}, yi = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const float br = lr[(4 * s + q) * 17 + c], bi = li[(4 * s + q) * 17 + c];
        yr = __builtin_amdgcn_mfma_f32_16x16x4f32(wr[s], br, yr, 0, 0, 0);
        yr = __builtin_amdgcn_mfma_f32_16x16x4f32(-wi[s], bi, yr, 0, 0, 0);
        yi = __builtin_amdgcn_mfma_f32_16x16x4f32(wr[s], bi, yi, 0, 0, 0);
        yi = __builtin_amdgcn_mfma_f32_16x16x4f32(wi[s], br, yi, 0, 0, 0);
    }
    return Cmat{yr, yi};
}

// Y = M Wx, M read from LDS as the A operand (W is symmetric: its B operand
// takes the same registers as its A operand)
__device__ __forceinline__ Cmat cm_times_w(const float* lr, const float* li, const float (&wr)[4],
                                           const float (&wi)[4], int q, int c)
{
    floatx4 yr = {0.f, 0.f, 0.f, 0.f}, yi = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const float ar = lr[c * 17 + 4 * s + q], ai = li[c * 17 + 4 * s + q];
        yr = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, wr[s], yr, 0, 0, 0);
        yr = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai, wi[s], yr, 0, 0, 0);
        yi = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, wi[s], yi, 0, 0, 0);
        yi = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, wr[s], yi, 0, 0, 0);
    }
    return Cmat{yr, yi};
}

// DFT on the matrix cores: one cell per wave.  With W[a][b] = exp(-2 pi i ab/16)
// (symmetric): H = f^T W (real input: two real products), O = W H with
// O[K1][K0] = fhat(K0, K1).  A round trip: H2 = conj(W) O, s^T = H2 conj(W) / n^2,
// H = s^T W, O = W H.
__global__ __launch_bounds__(256) void k_stage_dft16_mfma(int batch, int reps, const float* __restrict__ f,
                                                          float2* __restrict__ out)
{
    constexpr int N = 16, NPTS = N * N, LD = N + 1;
    __shared__ float lds[4][2][N * LD];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c = lane & 15, q = lane >> 4;
    // W[4s + q][c] for the four k-steps s (the lane's A and B operand of W)
    float wr[4], wi[4], wic[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int ph = ((4 * s + q) * c) & (N - 1);
        double sn, cs;
        sincos(-2.0 * M_PI * (double)ph / (double)N, &sn, &cs);
        wr[s] = (float)cs;
        wi[s] = (float)sn;
        wic[s] = -(float)sn;
    }
    float* lr = lds[wave][0];
    float* li = lds[wave][1];
    const int cells_per_grid = gridDim.x * 4;
    for (int cell = blockIdx.x * 4 + wave; cell < batch; cell += cells_per_grid) {
        const float* fc = f + (size_t)cell * NPTS;
        // A = f^T: lane l holds f[4s + q][c] = element 64 s + l
        float a[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) a[s] = fc[64 * s + lane];
        Cmat h;
        h.re = floatx4{0.f, 0.f, 0.f, 0.f};
        h.im = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            h.re = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], wr[s], h.re, 0, 0, 0);
            h.im = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], wi[s], h.im, 0, 0, 0);
        }
        cm_store(h, lr, li, q, c);
        wave_sync();
        Cmat o = cm_w_times(wr, wi, lr, li, q, c);
        for (int r = 0; r < reps; ++r) {
            wave_sync();
            cm_store(o, lr, li, q, c);
            wave_sync();
            Cmat h2 = cm_w_times(wr, wic, lr, li, q, c);
            wave_sync();
            cm_store(h2, lr, li, q, c);
            wave_sync();
            Cmat st = cm_times_w(lr, li, wr, wic, q, c);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                st.re[k] *= 1.f / NPTS;
                st.im[k] *= 1.f / NPTS;
            }
            wave_sync();
            cm_store(st, lr, li, q, c);
            wave_sync();
            Cmat hh = cm_times_w(lr, li, wr, wi, q, c);
            wave_sync();
            cm_store(hh, lr, li, q, c);
            wave_sync();
            o = cm_w_times(wr, wi, lr, li, q, c);
        }
        wave_sync();   // the next cell overwrites this wave's LDS rows
        float2* oc = out + (size_t)cell * NPTS;
#pragma unroll
        for (int r = 0; r < 4; ++r) oc[(4 * q + r) * N + c] = make_float2(o.re[r], o.im[r]);
    }
}

}  // namespace

hipError_t launch_transform_stage(int method, int batch, int reps, const float* f, float2* out, hipStream_t st)
{
    int grid = 0;
    hipError_t e;
    if (method == 0) {
        e = occupancy_grid(k_stage_fft16, 256, 0, (batch + 15) / 16, grid);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_stage_fft16, dim3(grid), dim3(256), 0, st, batch, reps, f, out);
    } else {
        e = occupancy_grid(k_stage_dft16_mfma, 256, 0, (batch + 3) / 4, grid);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_stage_dft16_mfma, dim3(grid), dim3(256), 0, st, batch, reps, f, out);
    }
    return hipGetLastError();
}

}  // namespace qdvm
