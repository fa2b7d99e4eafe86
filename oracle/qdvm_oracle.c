/*
 * qdvm_oracle.c -- plain FP64 CPU reference ("the oracle") for the fast
 * discrete-velocity (DVM) Boltzmann collision operator of Mouhot, Pareschi and
 * Rey, "Convolutive decomposition and fast summation methods for
 * discrete-velocity approximations of the Boltzmann equation".
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the GPU implementation; it enumerates its own
 * directions and evaluates the operator by direct summation, with no Fourier
 * transform anywhere.
 *
 * What it computes.  Sec. 2.3, eq. (2.9) defines the periodised, truncated DVM
 *
 *     D_i = sum_{-Nt <= k,l <= Nt} Gamma_{k,l} [ f_{i+k} f_{i+l} - f_i f_{i+k+l} ]
 *
 * with Gamma_{k,l} = 1(k.l) a(k) b(l) under the decoupling assumption of
 * Sec. 3.2, eq. (3.3).  The direction decomposition of Sec. 3.2, eqs.
 * (3.6)-(3.7), splits the sum over k != 0 by the lattice line e_p Z that k
 * lies on, and keeps only the lines of a chosen set {e_1..e_P}.  With the
 * weight a(k) constant along each line (the paper's a(k) = h^(2d-1)|k|/gcd(k)
 * equals h^(2d-1)|e_p|_2 for every k on the line of e_p) and b = 1, this is
 *
 *   Q_i = sum_p w_p sum_{0<|m|<=M_p} sum_{l in L_p}
 *                 [ f(i + m e_p) f(i + l) - f(i) f(i + m e_p + l) ]
 *
 *   M_p = floor(Nt / |e_p|_inf),   L_p = { l in Z^d : l.e_p = 0, |l|_inf <= Nt },
 *
 * on the periodic lattice (Z/nZ)^d (indices wrap mod n, Sec. 2.3).  Every
 * function also takes a line-weight profile: with line_weight = 1 the term of
 * k = m e_p carries w_p / |m| instead of w_p (a(k) = h^(2d-2)/gcd(k), the
 * lattice quadrature of delta(x . y) for a constant kernel).  The
 * vector-Jacobian product of Q with respect to f and to the weights w_p is
 * obtained by differentiating that sum term by term.
 *
 * Every function is a literal transcription of a sum: no factoring, blocking
 * or transform.  Grid points are flattened in C order (last axis fastest).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXD 3

/* ------------------------------------------------------------------------ */
/* Lattice lines (Sec. 3.2: Farey series, primal representatives of lines)  */
/* ------------------------------------------------------------------------ */

static int or_gcd(int a, int b)
{
    if (a < 0) a = -a;
    if (b < 0) b = -b;
    while (b) { int t = a % b; a = b; b = t; }
    return a;
}

static int or_abs(int a) { return a < 0 ? -a : a; }

static int or_norm_inf(int d, const int *e)
{
    int m = 0;
    for (int a = 0; a < d; ++a) if (or_abs(e[a]) > m) m = or_abs(e[a]);
    return m;
}

static int or_norm2sq(int d, const int *e)
{
    int s = 0;
    for (int a = 0; a < d; ++a) s += e[a] * e[a];
    return s;
}

/* Order key of a line: (|e|_inf, |e|_2^2, components ascending). */
static int or_line_cmp(int d, const int *x, const int *y)
{
    int a = or_norm_inf(d, x), b = or_norm_inf(d, y);
    if (a != b) return a < b ? -1 : 1;
    a = or_norm2sq(d, x); b = or_norm2sq(d, y);
    if (a != b) return a < b ? -1 : 1;
    for (int c = 0; c < d; ++c)
        if (x[c] != y[c]) return x[c] < y[c] ? -1 : 1;
    return 0;
}

/*
 * The lines through 0 of the box [-order, order]^d (the set A^{d-1} of
 * Sec. 3.2): one primitive vector per line (gcd of components 1), with its
 * first nonzero component positive, listed by the order key above.
 * Writes up to `cap` lines (d ints each) to `out`; returns the total count.
 */
int oracle_lines(int d, int order, int32_t *out, int cap)
{
    if (d < 2 || d > OR_MAXD || order < 1) return -1;
    int side = 2 * order + 1, total = 1;
    for (int a = 0; a < d; ++a) total *= side;
    int *buf = (int *)malloc(sizeof(int) * (size_t)total * d);
    int cnt = 0;
    for (int idx = 0; idx < total; ++idx) {
        int e[OR_MAXD], r = idx, g = 0, first = 0;
        for (int a = d - 1; a >= 0; --a) { e[a] = r % side - order; r /= side; }
        for (int a = 0; a < d; ++a) g = or_gcd(g, e[a]);
        if (g != 1) continue;                      /* zero vector or not primitive */
        for (int a = 0; a < d; ++a) if (e[a] != 0) { first = e[a]; break; }
        if (first < 0) continue;                   /* keep one sign per line */
        memcpy(buf + (size_t)cnt * d, e, sizeof(int) * d);
        ++cnt;
    }
    /* insertion sort by the order key (sizes here are at most a few thousand) */
    for (int i = 1; i < cnt; ++i) {
        int key[OR_MAXD];
        memcpy(key, buf + (size_t)i * d, sizeof(int) * d);
        int j = i - 1;
        while (j >= 0 && or_line_cmp(d, buf + (size_t)j * d, key) > 0) {
            memcpy(buf + (size_t)(j + 1) * d, buf + (size_t)j * d, sizeof(int) * d);
            --j;
        }
        memcpy(buf + (size_t)(j + 1) * d, key, sizeof(int) * d);
    }
    for (int i = 0; i < cnt && i < cap; ++i)
        for (int a = 0; a < d; ++a) out[(size_t)i * d + a] = buf[(size_t)i * d + a];
    free(buf);
    return cnt;
}

/*
 * Weights of Sec. 3.2 (after eq. (3.3)): a(k) = h^(2d-1) |k| / gcd(k), b = 1
 * (h^5 for 3D hard spheres, h^3 for 2D Maxwell molecules), with |k| measured
 * in lattice units.  For k = m e_p this is h^(2d-1) |e_p|_2 on the whole line.
 */
void oracle_default_weights(int d, double h, int P, const int32_t *dirs, int line_weight, double *w)
{
    /* uniform profile: h^(2d-1) |e_p|_2; delta profile: h^(2d-2) (then a(m e_p) = w_p / |m|) */
    double s = pow(h, 2 * d - 1);
    for (int p = 0; p < P; ++p) {
        double n2 = 0.0;
        for (int a = 0; a < d; ++a) n2 += (double)dirs[p * d + a] * dirs[p * d + a];
        w[p] = line_weight ? pow(h, 2 * d - 2) : s * sqrt(n2);
    }
}

/* ------------------------------------------------------------------------ */
/* Collision sets K_p, L_p                                                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    int nk, nl;
    int *k;     /* nk x d : m e_p, 0 < |m| <= M_p      */
    double *kw; /* nk     : weight factor of k = m e_p: 1 (uniform), 1/|m| (delta) */
    int *l;     /* nl x d : l.e_p = 0, |l|_inf <= Nt    */
} or_sets;

/*
 * Line-weight profile: a(k) for k = m e_p is w_p (line_weight 0, the paper's
 * lattice weight h^(2d-1)|k|/gcd(k), constant along a line) or w_p / |m|
 * (line_weight 1: the lattice quadrature of delta(x . y) for a constant
 * kernel, h^(2d-2)/gcd(k) with gcd(m e_p) = |m|).
 */
static void or_build_sets(int d, int ntilde, const int32_t *e, int line_weight, or_sets *s)
{
    int ninf = 0;
    for (int a = 0; a < d; ++a) if (or_abs(e[a]) > ninf) ninf = or_abs(e[a]);
    int M = ninf > 0 ? ntilde / ninf : 0;
    s->nk = 2 * M;
    s->k = (int *)malloc(sizeof(int) * (size_t)(s->nk > 0 ? s->nk : 1) * d);
    s->kw = (double *)malloc(sizeof(double) * (size_t)(s->nk > 0 ? s->nk : 1));
    int c = 0;
    for (int m = -M; m <= M; ++m) {
        if (m == 0) continue;
        for (int a = 0; a < d; ++a) s->k[c * d + a] = m * e[a];
        s->kw[c] = line_weight ? 1.0 / (double)or_abs(m) : 1.0;
        ++c;
    }
    int side = 2 * ntilde + 1, total = 1;
    for (int a = 0; a < d; ++a) total *= side;
    s->l = (int *)malloc(sizeof(int) * (size_t)total * d);
    s->nl = 0;
    for (int idx = 0; idx < total; ++idx) {
        int l[OR_MAXD], r = idx, dot = 0;
        for (int a = d - 1; a >= 0; --a) { l[a] = r % side - ntilde; r /= side; }
        for (int a = 0; a < d; ++a) dot += l[a] * e[a];
        if (dot != 0) continue;
        memcpy(s->l + (size_t)s->nl * d, l, sizeof(int) * d);
        s->nl++;
    }
}

static void or_free_sets(or_sets *s) { free(s->k); free(s->kw); free(s->l); }

/* flat index of (i + o) on the periodic grid, i given by its coordinates */
static inline long or_wrap(int d, int n, const int *i, const int *o1, const int *o2)
{
    long idx = 0;
    for (int a = 0; a < d; ++a) {
        int v = i[a] + o1[a] + (o2 ? o2[a] : 0);
        v %= n;
        if (v < 0) v += n;
        idx = idx * n + v;
    }
    return idx;
}

static inline void or_coords(int d, int n, long flat, int *i)
{
    for (int a = d - 1; a >= 0; --a) { i[a] = (int)(flat % n); flat /= n; }
}

static long or_npts(int d, int n)
{
    long t = 1;
    for (int a = 0; a < d; ++a) t *= n;
    return t;
}

/* ------------------------------------------------------------------------ */
/* The operator                                                              */
/* ------------------------------------------------------------------------ */

/*
 * Unit-weight contribution of each direction, Q_p (so that Q = sum_p w_p Q_p),
 * for one cell: qp[p * n^d + i].
 */
void oracle_collide_terms(int d, int n, int ntilde, int P, const int32_t *dirs, int line_weight,
                          const double *f, double *qp)
{
    long npts = or_npts(d, n);
    for (int p = 0; p < P; ++p) {
        or_sets s;
        or_build_sets(d, ntilde, dirs + (size_t)p * d, line_weight, &s);
        double *out = qp + (size_t)p * npts;
#pragma omp parallel for schedule(static)
        for (long flat = 0; flat < npts; ++flat) {
            int i[OR_MAXD];
            or_coords(d, n, flat, i);
            double acc = 0.0;
            for (int a = 0; a < s.nk; ++a) {
                const int *k = s.k + (size_t)a * d;
                long ik = or_wrap(d, n, i, k, NULL);
                for (int b = 0; b < s.nl; ++b) {
                    const int *l = s.l + (size_t)b * d;
                    long il = or_wrap(d, n, i, l, NULL);
                    long ikl = or_wrap(d, n, i, k, l);
                    acc += s.kw[a] * (f[ik] * f[il] - f[flat] * f[ikl]);
                }
            }
            out[flat] = acc;
        }
        or_free_sets(&s);
    }
}

/* Q = sum_p w_p Q_p for `batch` cells stored one after another. */
void oracle_collide(int d, int n, int ntilde, int P, const int32_t *dirs, const double *w, int line_weight,
                    int batch, const double *f, double *q)
{
    long npts = or_npts(d, n);
    or_sets *s = (or_sets *)malloc(sizeof(or_sets) * (size_t)(P > 0 ? P : 1));
    for (int p = 0; p < P; ++p) or_build_sets(d, ntilde, dirs + (size_t)p * d, line_weight, &s[p]);
    for (int cell = 0; cell < batch; ++cell) {
        const double *fc = f + (size_t)cell * npts;
        double *qc = q + (size_t)cell * npts;
#pragma omp parallel for schedule(static)
        for (long flat = 0; flat < npts; ++flat) {
            int i[OR_MAXD];
            or_coords(d, n, flat, i);
            double total = 0.0;
            for (int p = 0; p < P; ++p) {
                double acc = 0.0;
                for (int a = 0; a < s[p].nk; ++a) {
                    const int *k = s[p].k + (size_t)a * d;
                    long ik = or_wrap(d, n, i, k, NULL);
                    for (int b = 0; b < s[p].nl; ++b) {
                        const int *l = s[p].l + (size_t)b * d;
                        long il = or_wrap(d, n, i, l, NULL);
                        long ikl = or_wrap(d, n, i, k, l);
                        acc += s[p].kw[a] * (fc[ik] * fc[il] - fc[flat] * fc[ikl]);
                    }
                }
                total += w[p] * acc;
            }
            qc[flat] = total;
        }
    }
    for (int p = 0; p < P; ++p) or_free_sets(&s[p]);
    free(s);
}

/*
 * The bilinear operator of the consistency statement of Sec. 2.3 (Theorem
 * theo:HePa is stated for D(g, f)): eq. (2.9) with the two distribution
 * functions in the places the paper's Q(g, f) gives them -- g at the point
 * i + k of the gain and at i itself in the loss, f at i + l and i + k + l:
 *
 *   Q(g, f)_i = sum_p w_p sum_{k in K_p, l in L_p} [ g(i+k) f(i+l) - g(i) f(i+k+l) ]
 *
 * Q(f, f) is the diagonal.  Same sets and weights as oracle_collide.
 */
void oracle_collide_bilinear(int d, int n, int ntilde, int P, const int32_t *dirs, const double *w,
                             int line_weight, int batch, const double *g, const double *f, double *q)
{
    long npts = or_npts(d, n);
    or_sets *s = (or_sets *)malloc(sizeof(or_sets) * (size_t)(P > 0 ? P : 1));
    for (int p = 0; p < P; ++p) or_build_sets(d, ntilde, dirs + (size_t)p * d, line_weight, &s[p]);
    for (int cell = 0; cell < batch; ++cell) {
        const double *gc = g + (size_t)cell * npts;
        const double *fc = f + (size_t)cell * npts;
        double *qc = q + (size_t)cell * npts;
#pragma omp parallel for schedule(static)
        for (long flat = 0; flat < npts; ++flat) {
            int i[OR_MAXD];
            or_coords(d, n, flat, i);
            double total = 0.0;
            for (int p = 0; p < P; ++p) {
                double acc = 0.0;
                for (int a = 0; a < s[p].nk; ++a) {
                    const int *k = s[p].k + (size_t)a * d;
                    long ik = or_wrap(d, n, i, k, NULL);
                    for (int b = 0; b < s[p].nl; ++b) {
                        const int *l = s[p].l + (size_t)b * d;
                        long il = or_wrap(d, n, i, l, NULL);
                        long ikl = or_wrap(d, n, i, k, l);
                        acc += s[p].kw[a] * (gc[ik] * fc[il] - gc[flat] * fc[ikl]);
                    }
                }
                total += w[p] * acc;
            }
            qc[flat] = total;
        }
    }
    for (int p = 0; p < P; ++p) or_free_sets(&s[p]);
    free(s);
}

/*
 * Vector-Jacobian product.  With a cotangent c, the scalar <c, Q(f; w)> has
 *
 *   d/df_j : sum_p w_p sum_{k in K_p, l in L_p} ( c[j-k] f[j-k+l] + c[j-l] f[j-l+k]
 *                                               - c[j] f[j+k+l]   - c[j-k-l] f[j-k-l] )
 *   d/dw_p : sum_i c_i Q_p(i)
 *
 * (each bracket f_a f_b - f_c f_d of the sum differentiated by the index
 * substitution that puts the free index at j).  grad_w is summed over cells.
 */
void oracle_vjp(int d, int n, int ntilde, int P, const int32_t *dirs, const double *w, int line_weight,
                int batch, const double *f, const double *c, double *grad_f, double *grad_w)
{
    long npts = or_npts(d, n);
    or_sets *s = (or_sets *)malloc(sizeof(or_sets) * (size_t)(P > 0 ? P : 1));
    for (int p = 0; p < P; ++p) or_build_sets(d, ntilde, dirs + (size_t)p * d, line_weight, &s[p]);
    for (int p = 0; p < P; ++p) grad_w[p] = 0.0;
    double *qp = (double *)malloc(sizeof(double) * (size_t)npts * (P > 0 ? P : 1));
    for (int cell = 0; cell < batch; ++cell) {
        const double *fc = f + (size_t)cell * npts;
        const double *cc = c + (size_t)cell * npts;
        double *gc = grad_f + (size_t)cell * npts;
#pragma omp parallel for schedule(static)
        for (long flat = 0; flat < npts; ++flat) {
            int j[OR_MAXD];
            or_coords(d, n, flat, j);
            double total = 0.0;
            for (int p = 0; p < P; ++p) {
                double acc = 0.0;
                for (int a = 0; a < s[p].nk; ++a) {
                    const int *k = s[p].k + (size_t)a * d;
                    int mk[OR_MAXD];
                    for (int t = 0; t < d; ++t) mk[t] = -k[t];
                    long jmk = or_wrap(d, n, j, mk, NULL);
                    for (int b = 0; b < s[p].nl; ++b) {
                        const int *l = s[p].l + (size_t)b * d;
                        int ml[OR_MAXD];
                        for (int t = 0; t < d; ++t) ml[t] = -l[t];
                        long jmkpl = or_wrap(d, n, j, mk, l);   /* j-k+l */
                        long jml = or_wrap(d, n, j, ml, NULL);  /* j-l   */
                        long jmlpk = or_wrap(d, n, j, ml, k);   /* j-l+k */
                        long jpkl = or_wrap(d, n, j, k, l);     /* j+k+l */
                        long jmkml = or_wrap(d, n, j, mk, ml);  /* j-k-l */
                        acc += s[p].kw[a] * (cc[jmk] * fc[jmkpl] + cc[jml] * fc[jmlpk]
                                             - cc[flat] * fc[jpkl] - cc[jmkml] * fc[jmkml]);
                    }
                }
                total += w[p] * acc;
            }
            gc[flat] = total;
        }
        oracle_collide_terms(d, n, ntilde, P, dirs, line_weight, fc, qp);
        for (int p = 0; p < P; ++p) {
            double acc = 0.0;
            for (long i = 0; i < npts; ++i) acc += cc[i] * qp[(size_t)p * npts + i];
            grad_w[p] += acc;
        }
    }
    free(qp);
    for (int p = 0; p < P; ++p) or_free_sets(&s[p]);
    free(s);
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}
