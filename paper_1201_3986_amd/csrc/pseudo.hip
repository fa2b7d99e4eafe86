// The pseudo-spectral form of the discrete operator (Sec. 3.1): with the DFT
// f~ of f on the grid, Q~_I = sum_{K+L=I} beta~(K, L) f~_K f~_L, beta~(K, L) =
// beta(K, L) - beta(L, L) and the kernel modes beta(K, L) = sum over the
// collision pairs (k, l) of the weight times e_K(k) e_L(l) (eq. (3.2)).  Under
// the direction decomposition beta(K, L) = sum_p w_p alpha_p(K) alpha'_p(L),
// built on the host in FP64 (plan.cpp).  O(n^{2d}) per cell -- the cost the
// paper quotes for this form -- evaluated here by direct sums in FP64: a
// second, independent GPU evaluation of Q(f, f) for small grids, against
// which the fast FP32 path can be checked on the device.
#include "kernels_common.h"

namespace qdvm {

namespace {

// One workgroup of 256 threads per cell, persistent over cells.  LDS: f, its
// DFT and the DFT of Q (FP64), and the n roots of unity.
__global__ __launch_bounds__(256) void k_pseudo(int dim, int n, int npts, int batch, const double* __restrict__ beta,
                                                const float* __restrict__ f, float* __restrict__ q)
{
    extern __shared__ double sm[];
    double* fv = sm;                       // [npts]
    double* fr = fv + npts;                // [npts] Re fhat
    double* fi = fr + npts;                // [npts] Im fhat
    double* qr = fi + npts;                // [npts] Re Qhat
    double* qi = qr + npts;                // [npts] Im Qhat
    double* cs = qi + npts;                // [n] cos(2 pi r / n)
    double* sn = cs + n;                   // [n] sin(2 pi r / n)
    const int tid = threadIdx.x;
    for (int r = tid; r < n; r += 256) sincospi(2.0 * r / n, &sn[r], &cs[r]);
    const double inv2 = 1.0 / ((double)npts * (double)npts);
    auto coord = [&](int idx, int* c) {
        for (int a = dim - 1; a >= 0; --a) {
            c[a] = idx % n;
            idx /= n;
        }
    };
    for (int cell = blockIdx.x; cell < batch; cell += gridDim.x) {
        __syncthreads();
        for (int i = tid; i < npts; i += 256) fv[i] = (double)f[(size_t)cell * npts + i];
        __syncthreads();
        // fhat_K = sum_j f_j exp(-2 pi i K.j / n)
        for (int K = tid; K < npts; K += 256) {
            int kc[3];
            coord(K, kc);
            double re = 0.0, im = 0.0;
            for (int j = 0; j < npts; ++j) {
                int jc[3];
                coord(j, jc);
                int ph = 0;
                for (int a = 0; a < dim; ++a) ph += kc[a] * jc[a];
                ph %= n;
                re += fv[j] * cs[ph];
                im -= fv[j] * sn[ph];
            }
            fr[K] = re;
            fi[K] = im;
        }
        __syncthreads();
        // Qhat_I = sum_K beta~(K, I - K) fhat_K fhat_{I-K} / n^{2d}
        for (int I = tid; I < npts; I += 256) {
            int ic[3];
            coord(I, ic);
            double re = 0.0, im = 0.0;
            for (int K = 0; K < npts; ++K) {
                int kc[3];
                coord(K, kc);
                int L = 0;
                for (int a = 0; a < dim; ++a) L = L * n + (ic[a] - kc[a] + n) % n;
                const double b = beta[(size_t)K * npts + L];
                re += b * (fr[K] * fr[L] - fi[K] * fi[L]);
                im += b * (fr[K] * fi[L] + fi[K] * fr[L]);
            }
            qr[I] = re * inv2;
            qi[I] = im * inv2;
        }
        __syncthreads();
        // Q_j = Re sum_I Qhat_I exp(2 pi i I.j / n)
        for (int j = tid; j < npts; j += 256) {
            int jc[3];
            coord(j, jc);
            double re = 0.0;
            for (int I = 0; I < npts; ++I) {
                int ic[3];
                coord(I, ic);
                int ph = 0;
                for (int a = 0; a < dim; ++a) ph += ic[a] * jc[a];
                ph %= n;
                re += qr[I] * cs[ph] - qi[I] * sn[ph];
            }
            q[(size_t)cell * npts + j] = (float)re;
        }
    }
}

}  // namespace

hipError_t launch_pseudo(int dim, int n, int batch, const double* beta, const float* f, float* q, hipStream_t st)
{
    int npts = 1;
    for (int a = 0; a < dim; ++a) npts *= n;
    const size_t lds = sizeof(double) * (5 * (size_t)npts + 2 * (size_t)n);
    int grid = 0;
    hipError_t e = occupancy_grid(k_pseudo, 256, lds, batch, grid);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pseudo, dim3(grid), dim3(256), lds, st, dim, n, npts, batch, beta, f, q);
    return hipGetLastError();
}

}  // namespace qdvm
