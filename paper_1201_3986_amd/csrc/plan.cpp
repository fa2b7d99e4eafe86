// Host-side plan construction for the fast DVM collision operator:
// direction set, line lengths, weights, transform jobs and the FP64-built
// spectral multiplier tables (rounded once to FP32 for the device).
//
// References are to Mouhot, Pareschi, Rey, "Convolutive decomposition and fast
// summation methods for discrete-velocity approximations of the Boltzmann
// equation".
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <numeric>
#include <set>
#include <tuple>

#include "qdvm_internal.h"

namespace qdvm {

bool supported_size(int dim, int n)
{
    if (dim == 2) return n == 8 || n == 16 || n == 32 || n == 64;
    if (dim == 3) return n == 8 || n == 16 || n == 24 || n == 32;
    return false;
}

namespace {

int igcd(int a, int b)
{
    a = std::abs(a);
    b = std::abs(b);
    while (b) {
        int t = a % b;
        a = b;
        b = t;
    }
    return a;
}

using Line = std::vector<int32_t>;

// Canonical order of lines: (|e|_inf, |e|_2^2, components ascending).
bool line_less(const Line& a, const Line& b)
{
    auto key = [](const Line& e) {
        int inf = 0, n2 = 0;
        for (int x : e) {
            inf = std::max(inf, std::abs(x));
            n2 += x * x;
        }
        return std::make_tuple(inf, n2);
    };
    auto ka = key(a), kb = key(b);
    if (ka != kb) return ka < kb;
    return a < b;
}

// Lines through 0 of [-order, order]^dim (the set A^{dim-1} of Sec. 3.2), one
// primitive vector per line with first nonzero component positive.  Built shell
// by shell in |e|_inf so that the first P lines of a larger order coincide.
std::vector<Line> lines_of_order(int dim, int order)
{
    std::vector<Line> out;
    for (int shell = 1; shell <= order; ++shell) {
        std::vector<Line> sh;
        int side = 2 * shell + 1;
        int total = 1;
        for (int a = 0; a < dim; ++a) total *= side;
        for (int idx = 0; idx < total; ++idx) {
            Line e(dim);
            int r = idx, inf = 0, g = 0;
            for (int a = dim - 1; a >= 0; --a) {
                e[a] = r % side - shell;
                r /= side;
            }
            for (int x : e) {
                inf = std::max(inf, std::abs(x));
                g = igcd(g, x);
            }
            if (inf != shell || g != 1) continue;
            int first = 0;
            for (int x : e)
                if (x) {
                    first = x;
                    break;
                }
            if (first < 0) continue;
            sh.push_back(e);
        }
        std::sort(sh.begin(), sh.end(), line_less);
        out.insert(out.end(), sh.begin(), sh.end());
    }
    return out;
}

}  // namespace

std::string build_host_plan(int dim, int n, double half_width, int ntilde, int farey_order,
                            int num_dirs, const int32_t* dirs, const double* weights, int line_weight, HostPlan& hp)
{
    char msg[256];
    if (dim != 2 && dim != 3) return "invalid: dim must be 2 or 3";
    if (line_weight != 0 && line_weight != 1)
        return "invalid: line_weight must be QDVM_LINE_UNIFORM (0) or QDVM_LINE_DELTA (1)";
    if (n < 2) return "invalid: n must be at least 2";
    if (!supported_size(dim, n)) {
        std::snprintf(msg, sizeof msg, "unsupported: n = %d for dim %d (2D: 8,16,32,64; 3D: 8,16,24,32)", n, dim);
        return msg;
    }
    if (!(half_width > 0.0) || !std::isfinite(half_width)) return "invalid: half_width must be positive and finite";
    // Default truncation Nt = floor(n / (3 + sqrt 2)) (Sec. 4, next to Table 1).
    if (ntilde == 0) ntilde = (int)std::floor(n / (3.0 + std::sqrt(2.0)));
    if (ntilde < 1 || 2 * ntilde + 1 > n) {
        std::snprintf(msg, sizeof msg, "invalid: ntilde = %d needs 1 <= ntilde and 2*ntilde+1 <= n = %d", ntilde, n);
        return msg;
    }
    std::vector<Line> L;
    if (dirs) {
        if (num_dirs < 1 || num_dirs > 65536) return "invalid: num_dirs must be in [1, 65536] with explicit dirs";
        std::set<Line> seen;
        for (int p = 0; p < num_dirs; ++p) {
            Line e(dirs + (size_t)p * dim, dirs + (size_t)(p + 1) * dim);
            int g = 0, first = 0;
            for (int x : e) {
                g = igcd(g, x);
                if (!first && x) first = x;
                if (std::abs(x) > 1 << 20) return "invalid: direction component too large";
            }
            if (g != 1) {
                std::snprintf(msg, sizeof msg, "invalid: direction %d is zero or not primitive", p);
                return msg;
            }
            if (first < 0) {
                std::snprintf(msg, sizeof msg, "invalid: direction %d must have its first nonzero component positive", p);
                return msg;
            }
            if (!seen.insert(e).second) {
                std::snprintf(msg, sizeof msg, "invalid: direction %d duplicates an earlier line", p);
                return msg;
            }
            L.push_back(e);
        }
    } else if (num_dirs > 0) {
        if (num_dirs > 65536) return "invalid: num_dirs too large";
        int order = 1;
        for (;;) {
            L = lines_of_order(dim, order);
            if ((int)L.size() >= num_dirs) break;
            ++order;
        }
        L.resize(num_dirs);
    } else if (farey_order >= 1) {
        if (farey_order > 64) return "invalid: farey_order too large (max 64)";
        L = lines_of_order(dim, farey_order);
    } else {
        return "invalid: give dirs, num_dirs > 0 or farey_order >= 1";
    }

    hp.dim = dim;
    hp.n = n;
    hp.line_weight = line_weight;
    hp.ntilde = ntilde;
    hp.half_width = half_width;
    hp.h = 2.0 * half_width / n;
    hp.P = (int)L.size();
    hp.dirs.clear();
    hp.M.clear();
    hp.weights.assign(hp.P, 0.0);
    for (int p = 0; p < hp.P; ++p) {
        int inf = 0;
        double n2 = 0;
        for (int x : L[p]) {
            hp.dirs.push_back(x);
            inf = std::max(inf, std::abs(x));
            n2 += double(x) * x;
        }
        hp.M.push_back(ntilde / inf);
        // uniform profile: a(k) = h^(2d-1) |k| / gcd(k) (Sec. 3.2, after eq. (3.3)), constant on
        // a line; delta profile: a(m e_p) = w_p / |m| with w_p = h^(2d-2), the lattice quadrature
        // of delta(x . y) for a constant kernel
        const double wdef = line_weight ? std::pow(hp.h, 2 * dim - 2) : std::pow(hp.h, 2 * dim - 1) * std::sqrt(n2);
        hp.weights[p] = weights ? weights[p] : wdef;
        if (weights && !std::isfinite(weights[p])) return "invalid: weights must be finite";
    }

    // Jobs: one inverse transform per direction with M >= 1; in 2D a direction
    // and its perpendicular share one (their unit-weight terms are equal only
    // when the weight is uniform along the line, Remark 3.5).
    hp.jobs.clear();
    std::vector<int> used(hp.P, 0);
    for (int p = 0; p < hp.P; ++p) {
        if (hp.M[p] < 1 || used[p]) continue;
        JobDesc j{};
        for (int a = 0; a < dim; ++a) j.e[a] = L[p][a];
        j.M = hp.M[p];
        j.p = p;
        j.pp = -1;
        used[p] = 1;
        if (dim == 2 && line_weight == 0) {
            Line perp = {-L[p][1], L[p][0]};
            if (perp[0] < 0 || (perp[0] == 0 && perp[1] < 0)) perp = {L[p][1], -L[p][0]};
            for (int r = p + 1; r < hp.P; ++r)
                if (!used[r] && L[r] == perp) {
                    j.pp = r;
                    used[r] = 1;
                    break;
                }
        }
        hp.jobs.push_back(j);
    }
    hp.dir_job.assign(hp.P, -1);
    for (size_t jb = 0; jb < hp.jobs.size(); ++jb) {
        hp.dir_job[hp.jobs[jb].p] = (int32_t)jb;
        if (hp.jobs[jb].pp >= 0) hp.dir_job[hp.jobs[jb].pp] = (int32_t)jb;
    }

    // Multiplier rows, M = 0..Nt, built in FP64 with the phase m*s reduced mod n
    // in integers: first the Dirichlet kernel D_M(s) = sum_{|m|<=M} cos(2 pi m s / n)
    // (the 2D plane sum), then the line multipliers
    // A_M(s) = sum_{0<|m|<=M} rho(m) cos(2 pi m s / n), rho = 1 (uniform profile,
    // A_M = D_M - 1) or 1/|m| (delta profile).
    std::vector<double> ct(n);
    for (int r = 0; r < n; ++r) ct[r] = std::cos(2.0 * M_PI * r / n);
    const size_t rows = (size_t)(ntilde + 1) * n;
    hp.dirichlet.assign(2 * rows, 0.f);
    for (int M = 0; M <= ntilde; ++M)
        for (int s = 0; s < n; ++s) {
            double d = 1.0, a = 0.0;
            for (int m = 1; m <= M; ++m) {
                d += 2.0 * ct[(m * s) % n];
                a += 2.0 * ct[(m * s) % n] / (line_weight ? (double)m : 1.0);
            }
            hp.dirichlet[(size_t)M * n + s] = (float)d;
            hp.dirichlet[rows + (size_t)M * n + s] = (float)a;
        }

    // 3D plane multipliers alpha'_p(K) = sum_{l.e_p = 0, |l|_inf <= Nt} cos(2 pi K.l / n)
    // (Sec. 3.2, after eq. (3.6)), stored in the spectral pencil layout
    // idx = Kz*n^2 + Kx*n + Ky.
    hp.aperp.clear();
    if (dim == 3) {
        const int npts = n * n * n;
        hp.aperp.assign((size_t)hp.jobs.size() * npts, 0.f);
        const int side = 2 * ntilde + 1;
        for (size_t jb = 0; jb < hp.jobs.size(); ++jb) {
            const JobDesc& J = hp.jobs[jb];
            std::vector<std::array<int, 3>> pl;
            for (int a = -ntilde; a <= ntilde; ++a)
                for (int b = -ntilde; b <= ntilde; ++b)
                    for (int c = -ntilde; c <= ntilde; ++c)
                        if (a * J.e[0] + b * J.e[1] + c * J.e[2] == 0) pl.push_back({a, b, c});
            (void)side;
            // the multiplier depends on K only through K mod n; sum over the plane set
            for (int kz = 0; kz < n; ++kz)
                for (int kx = 0; kx < n; ++kx)
                    for (int ky = 0; ky < n; ++ky) {
                        double acc = 0.0;
                        for (const auto& l : pl) {
                            int r = (kx * l[0] + ky * l[1] + kz * l[2]) % n;
                            if (r < 0) r += n;
                            acc += ct[r];
                        }
                        hp.aperp[jb * npts + (size_t)kz * n * n + kx * n + ky] = (float)acc;
                    }
        }
    }
    return std::string();
}

bool pseudo_supported(int dim, int n) { return (dim == 2 && n <= 32) || (dim == 3 && n == 8); }

// Kernel modes of the pseudo-spectral form (Sec. 3.1, eq. (3.2)) under the
// direction decomposition: beta(K, L) = sum_p w_p alpha_p(K) alpha'_p(L) with
// the line multiplier alpha_p(K) = sum_{0<|m|<=M_p} rho(m) cos(2 pi m e_p.K / n)
// and the plane multiplier alpha'_p(L) = sum_{l.e_p = 0, |l|_inf <= Nt} cos(2 pi L.l / n);
// beta~(K, L) = beta(K, L) - beta(L, L).  Indices in C order.
std::vector<double> build_pseudo_modes(const HostPlan& hp)
{
    const int d = hp.dim, n = hp.n, nt = hp.ntilde;
    int npts = 1;
    for (int a = 0; a < d; ++a) npts *= n;
    std::vector<double> ct(n);
    for (int r = 0; r < n; ++r) ct[r] = std::cos(2.0 * M_PI * r / n);
    auto coord = [&](int idx, int* c) {
        for (int a = d - 1; a >= 0; --a) {
            c[a] = idx % n;
            idx /= n;
        }
    };
    std::vector<double> beta((size_t)npts * npts, 0.0), al(npts), ap(npts);
    for (int p = 0; p < hp.P; ++p) {
        const int M = hp.M[p];
        if (M < 1) continue;
        const int* e = &hp.dirs[(size_t)p * d];
        std::vector<std::array<int, 3>> plane;
        const int side = 2 * nt + 1;
        int total = 1;
        for (int a = 0; a < d; ++a) total *= side;
        for (int idx = 0; idx < total; ++idx) {
            std::array<int, 3> l{0, 0, 0};
            int r = idx, dot = 0;
            for (int a = d - 1; a >= 0; --a) {
                l[a] = r % side - nt;
                r /= side;
            }
            for (int a = 0; a < d; ++a) dot += l[a] * e[a];
            if (dot == 0) plane.push_back(l);
        }
        for (int K = 0; K < npts; ++K) {
            int kc[3] = {0, 0, 0};
            coord(K, kc);
            int s = 0;
            for (int a = 0; a < d; ++a) s += e[a] * kc[a];
            s = ((s % n) + n) % n;
            double A = 0.0;
            for (int m = 1; m <= M; ++m) A += 2.0 * ct[(m * s) % n] / (hp.line_weight ? (double)m : 1.0);
            al[K] = A;
            double B = 0.0;
            for (const auto& l : plane) {
                int t = 0;
                for (int a = 0; a < d; ++a) t += kc[a] * l[a];
                B += ct[((t % n) + n) % n];
            }
            ap[K] = B;
        }
        const double w = (double)(float)hp.weights[p];
        for (int K = 0; K < npts; ++K) {
            const double wa = w * al[K];
            double* row = &beta[(size_t)K * npts];
            for (int L = 0; L < npts; ++L) row[L] += wa * ap[L];
        }
    }
    std::vector<double> diag(npts);
    for (int L = 0; L < npts; ++L) diag[L] = beta[(size_t)L * npts + L];
    for (int K = 0; K < npts; ++K)
        for (int L = 0; L < npts; ++L) beta[(size_t)K * npts + L] -= diag[L];
    return beta;
}

}  // namespace qdvm
