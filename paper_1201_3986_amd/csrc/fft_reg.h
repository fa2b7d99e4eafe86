// In-register FFTs for one lane, fully unrolled, for the small lengths the
// collision kernels use (8, 16, 24, 32, 64).
//
// A lane owns a whole pencil of N complex values in VGPRs.  The transform is a
// mixed-radix decimation-in-frequency sweep (radices given as a template pack,
// first radix applied first), which leaves the spectrum in digit-reversed
// order; the final reordering is a compile-time renaming of registers and
// costs no instruction.  Twiddles are compile-time constants computed in
// double precision by exact integer octant reduction followed by a Taylor
// series, then rounded once to float.
//
// Sign convention: SIGN = -1 computes X_k = sum_n x_n exp(-2 pi i n k / N)
// (forward), SIGN = +1 the unnormalised inverse.
#pragma once
#include <hip/hip_runtime.h>

namespace qdvm {

// ---------------------------------------------------------------- constants
constexpr double kPi = 3.141592653589793238462643383279502884;

constexpr double taylor_sin(double x)  // |x| <= pi/4
{
    double x2 = x * x, term = x, sum = x;
    for (int i = 1; i < 16; ++i) {
        term *= -x2 / double((2 * i) * (2 * i + 1));
        sum += term;
    }
    return sum;
}

constexpr double taylor_cos(double x)  // |x| <= pi/4
{
    double x2 = x * x, term = 1.0, sum = 1.0;
    for (int i = 1; i < 16; ++i) {
        term *= -x2 / double((2 * i - 1) * (2 * i));
        sum += term;
    }
    return sum;
}

// cos and sin of 2 pi k / N with the quadrant and octant taken in integers.
constexpr void cis2pi(long k, long N, double& c, double& s)
{
    k %= N;
    if (k < 0) k += N;
    long q = (4 * k) / N;        // quadrant
    long r = 4 * k - q * N;      // angle within quadrant = (pi/2) r / N, r in [0, N)
    double cq = 0, sq = 0;
    if (2 * r <= N) {
        double phi = (kPi / 2) * double(r) / double(N);
        cq = taylor_cos(phi);
        sq = taylor_sin(phi);
    } else {
        double phi = (kPi / 2) * double(N - r) / double(N);
        cq = taylor_sin(phi);
        sq = taylor_cos(phi);
    }
    switch (q) {
        case 0: c = cq; s = sq; break;
        case 1: c = -sq; s = cq; break;
        case 2: c = -cq; s = -sq; break;
        default: c = sq; s = -cq; break;
    }
}

template <int N>
struct TwTable {
    float c[N];
    float s[N];
    constexpr TwTable() : c(), s()
    {
        for (int k = 0; k < N; ++k) {
            double cc = 0, ss = 0;
            cis2pi(k, N, cc, ss);
            c[k] = float(cc);
            s[k] = float(ss);
        }
    }
};

template <int N>
inline constexpr TwTable<N> kTw{};

// ---------------------------------------------------------------- complex ops
__host__ __device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(__builtin_fmaf(a.x, b.x, -a.y * b.y), __builtin_fmaf(a.x, b.y, a.y * b.x));
}
// multiply by SIGN * i
template <int SIGN>
__host__ __device__ __forceinline__ float2 mul_si(float2 a)
{
    return SIGN > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// multiply by exp(SIGN * 2 pi i t / N), exact for multiples of a quarter turn
template <int N, int SIGN>
__host__ __device__ __forceinline__ float2 twiddle_mul(float2 a, int t)
{
    t %= N;
    if (t == 0) return a;
    if ((4 * t) % N == 0) {
        int q = (4 * t) / N;
        if (q == 2) return make_float2(-a.x, -a.y);
        return q == 1 ? mul_si<SIGN>(a) : mul_si<-SIGN>(a);
    }
    const float c = kTw<N>.c[t];
    const float s = SIGN > 0 ? kTw<N>.s[t] : -kTw<N>.s[t];
    return cmul(a, make_float2(c, s));
}

// ---------------------------------------------------------------- small DFTs
template <int R, int SIGN>
struct Dft;

template <int SIGN>
struct Dft<2, SIGN> {
    static __host__ __device__ __forceinline__ void run(float2* y)
    {
        float2 a = y[0], b = y[1];
        y[0] = cadd(a, b);
        y[1] = csub(a, b);
    }
};

template <int SIGN>
struct Dft<3, SIGN> {
    static __host__ __device__ __forceinline__ void run(float2* y)
    {
        constexpr float h = 0.8660254037844386f;  // sin(2 pi / 3)
        float2 t = cadd(y[1], y[2]);
        float2 u = csub(y[1], y[2]);
        float2 m = make_float2(__builtin_fmaf(-0.5f, t.x, y[0].x), __builtin_fmaf(-0.5f, t.y, y[0].y));
        float2 r = mul_si<SIGN>(make_float2(h * u.x, h * u.y));
        y[0] = cadd(y[0], t);
        y[1] = cadd(m, r);
        y[2] = csub(m, r);
    }
};

template <int SIGN>
struct Dft<4, SIGN> {
    static __host__ __device__ __forceinline__ void run(float2* y)
    {
        float2 t0 = cadd(y[0], y[2]), t1 = csub(y[0], y[2]);
        float2 t2 = cadd(y[1], y[3]), t3 = mul_si<SIGN>(csub(y[1], y[3]));
        y[0] = cadd(t0, t2);
        y[2] = csub(t0, t2);
        y[1] = cadd(t1, t3);
        y[3] = csub(t1, t3);
    }
};

template <int SIGN>
struct Dft<8, SIGN> {
    static __host__ __device__ __forceinline__ void run(float2* y)
    {
        constexpr float r2 = 0.70710678118654752f;
        float2 e[4] = {y[0], y[2], y[4], y[6]};
        float2 o[4] = {y[1], y[3], y[5], y[7]};
        Dft<4, SIGN>::run(e);
        Dft<4, SIGN>::run(o);
        // o[k] *= exp(SIGN i pi k / 4)
        float2 o1 = make_float2(r2 * (o[1].x - SIGN * o[1].y), r2 * (o[1].y + SIGN * o[1].x));
        float2 o2 = mul_si<SIGN>(o[2]);
        float2 o3 = make_float2(r2 * (-o[3].x - SIGN * o[3].y), r2 * (-o[3].y + SIGN * o[3].x));
        y[0] = cadd(e[0], o[0]);
        y[4] = csub(e[0], o[0]);
        y[1] = cadd(e[1], o1);
        y[5] = csub(e[1], o1);
        y[2] = cadd(e[2], o2);
        y[6] = csub(e[2], o2);
        y[3] = cadd(e[3], o3);
        y[7] = csub(e[3], o3);
    }
};

// ---------------------------------------------------------------- DIF sweep
template <int N, int SIGN, int L, int... Rs>
struct DifStages {
    static __host__ __device__ __forceinline__ void run(float2*) {}
};

template <int N, int SIGN, int L, int R, int... Rs>
struct DifStages<N, SIGN, L, R, Rs...> {
    static_assert(L % R == 0, "radix does not divide the block length");
    static __host__ __device__ __forceinline__ void run(float2* x)
    {
        constexpr int M = L / R;
#pragma unroll
        for (int b = 0; b < N; b += L) {
#pragma unroll
            for (int j = 0; j < M; ++j) {
                float2 y[R];
#pragma unroll
                for (int n0 = 0; n0 < R; ++n0) y[n0] = x[b + n0 * M + j];
                Dft<R, SIGN>::run(y);
#pragma unroll
                for (int k0 = 0; k0 < R; ++k0)
                    x[b + k0 * M + j] = twiddle_mul<N, SIGN>(y[k0], j * k0 * (N / L));
            }
        }
        DifStages<N, SIGN, M, Rs...>::run(x);
    }
};

// position of spectral index k after the DIF sweep with radices Rs...
template <int L, int... Rs>
struct DigitRev {
    static constexpr int pos(int) { return 0; }
};
template <int L, int R, int... Rs>
struct DigitRev<L, R, Rs...> {
    static constexpr int pos(int k) { return (k % R) * (L / R) + DigitRev<L / R, Rs...>::pos(k / R); }
};

template <int... Rs>
struct RadixProduct {
    static constexpr int value = (1 * ... * Rs);
};

// In-place FFT of one pencil held in registers, natural order in and out.
template <int N, int SIGN, int... Rs>
__host__ __device__ __forceinline__ void fft_pencil(float2 (&x)[N])
{
    static_assert(RadixProduct<Rs...>::value == N, "radices must multiply to N");
    DifStages<N, SIGN, N, Rs...>::run(x);
    float2 t[N];
#pragma unroll
    for (int k = 0; k < N; ++k) t[k] = x[DigitRev<N, Rs...>::pos(k)];
#pragma unroll
    for (int k = 0; k < N; ++k) x[k] = t[k];
}

// Default radix choice per length (the autotuner may override).
template <int N, int VARIANT>
struct Radix;
template <> struct Radix<8, 0> { template <int S> static __host__ __device__ __forceinline__ void fft(float2 (&x)[8]) { fft_pencil<8, S, 8>(x); } };
template <> struct Radix<8, 1> { template <int S> static __host__ __device__ __forceinline__ void fft(float2 (&x)[8]) { fft_pencil<8, S, 2, 4>(x); } };
template <> struct Radix<16, 0> { template <int S> static __host__ __device__ __forceinline__ void fft(float2 (&x)[16]) { fft_pencil<16, S, 4, 4>(x); } };
template <> struct Radix<16, 1> { template <int S> static __host__ __device__ __forceinline__ void fft(float2 (&x)[16]) { fft_pencil<16, S, 8, 2>(x); } };
template <> struct Radix<24, 0> { template <int S> static __host__ __device__ __forceinline__ void fft(float2 (&x)[24]) { fft_pencil<24, S, 8, 3>(x); } };
template <> struct Radix<24, 1> { template <int S> static __host__ __device__ __forceinline__ void fft(float2 (&x)[24]) { fft_pencil<24, S, 3, 8>(x); } };
template <> struct Radix<32, 0> { template <int S> static __host__ __device__ __forceinline__ void fft(float2 (&x)[32]) { fft_pencil<32, S, 8, 4>(x); } };
template <> struct Radix<32, 1> { template <int S> static __host__ __device__ __forceinline__ void fft(float2 (&x)[32]) { fft_pencil<32, S, 4, 8>(x); } };
template <> struct Radix<64, 0> { template <int S> static __host__ __device__ __forceinline__ void fft(float2 (&x)[64]) { fft_pencil<64, S, 8, 8>(x); } };
template <> struct Radix<64, 1> { template <int S> static __host__ __device__ __forceinline__ void fft(float2 (&x)[64]) { fft_pencil<64, S, 4, 4, 4>(x); } };

}  // namespace qdvm
