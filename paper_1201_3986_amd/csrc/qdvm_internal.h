// Internal types shared by the host plan builder and the HIP kernels of the
// qdvm library.  Nothing here is part of the public C interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qdvm.h"

#include <string>
#include <vector>

namespace qdvm {

// 2D evaluation with more jobs than this flushes its FP32 gain accumulator
// every kFlushJobs jobs into a compensated sum in scratch memory (cells_2d.h).
constexpr int kFlushJobs = 8;
// LDS of one workgroup on gfx950 (bytes).
constexpr size_t kMaxLds = 160 * 1024;

// One inverse transform of the direction loop ("job").  In 2D a line e and its
// perpendicular e' give the same unit-weight term (Remark 3.5), so a job may
// carry two directions, whose weights are added.
struct JobDesc {
    int32_t e[3];   // primitive representative (third component 0 in 2D)
    int32_t M;      // floor(Nt / |e|_inf) >= 1: the line sum runs over 0 < |m| <= M
    int32_t p;      // direction index in the plan
    int32_t pp;     // paired perpendicular direction, or -1
};

// LDS floats of a 2D plan's per-job multiplier tables (the layout of
// build_job_table in cells_2d.h): per job, a table for the line walk of
// stride e1 and one for the plane walk of stride e0; a stride d = 0 mod n
// takes n floats, else n + gcd(d, n) n (n a power of two).
inline int jt_table_floats(const JobDesc* jobs, int njobs, int n)
{
    auto size = [n](int e) {
        const int d = ((e % n) + n) % n;
        return d == 0 ? n : n + (d & -d) * n;
    };
    int t = 0;
    for (int jb = 0; jb < njobs; ++jb) t += size(jobs[jb].e[1]) + size(jobs[jb].e[0]);
    return t;
}

// Device view of an immutable plan, passed to kernels by value.
struct DevPlan {
    int32_t dim, n, ntilde, P, njobs;
    int32_t npts;                // n^dim
    int32_t mode;                // 0: Q(f, f); 1: near-equilibrium Q(f, f) - Q(M, M)
    const JobDesc* jobs;         // [njobs]
    const float* dirichlet;      // [2 (ntilde+1) n]: rows D_M(s) = sum_{|m|<=M} cos(2 pi m s / n), then the
                                 // line multipliers A_M(s) = sum_{0<|m|<=M} rho(m) cos(2 pi m s / n)
    const float* aperp;          // 3D: [njobs][npts] plane multipliers, spectral layout; 2D: null
    const float* w_default;      // [P] default weights
    const int32_t* dir_job;      // [P] job holding each direction, -1 if M_p = 0
    const float* lam0;           // [npts] Lambda / npts for the default weights
    const float* jobw0;          // [njobs] job weights / npts^2 for the default weights
    const float* lamb0;          // [npts] Lambda / npts of the bilinear operator (directions unpaired)
    const float* dirw0;          // [P] direction weights / npts^2 for the default weights
    int32_t jt_floats;           // 2D: LDS floats of the per-job multiplier tables (cells_2d.h)
};

// Per-call scratch carved out of a plan's workspace.
struct DevScratch {
    float* lam;      // [npts]  loss multiplier Lambda / npts, spectral layout
    float* jobw;     // [njobs] combined job weight / npts^2
    float2* spec;    // [slots * npts] spectrum of f per resident cell slot
    float2* spec2;   // [slots * npts] second spectral buffer (adjoint; g in near-equilibrium mode)
    float2* acc;     // [slots * npts] spectral accumulator (adjoint)
    double* gw_part; // [rows][njobs] FP64 job partials of grad_w (adjoint): one row per resident
                     // slot, accumulating that slot's cells in launch order (persistent launches),
                     // or one row per cell (direction-split launches); rows = min(batch, slots)
    float* part;     // [jsplit][batch][npts] per-workgroup parts of Q or grad_f (direction-split launches)
    int32_t* counter;  // work-queue counter (batched)
};

struct HostPlan {
    int32_t dim = 0, n = 0, ntilde = 0, P = 0, mode = 0;
    int32_t line_weight = 0;          // 0: uniform along a line; 1: 1/|m| (delta quadrature)
    double half_width = 0, h = 0;
    std::vector<int32_t> dirs;       // P * dim
    std::vector<double> weights;     // P
    std::vector<int32_t> M;          // P
    std::vector<JobDesc> jobs;
    std::vector<float> dirichlet;    // 2 (ntilde+1) n: D_M rows, then A_M rows
    std::vector<float> aperp;        // njobs * npts (3D)
    // device copies
    JobDesc* d_jobs = nullptr;
    float* d_dirichlet = nullptr;
    float* d_aperp = nullptr;
    float* d_w = nullptr;
    int32_t* d_dir_job = nullptr;
    float* d_lam0 = nullptr;
    float* d_jobw0 = nullptr;
    float* d_lamb0 = nullptr;
    float* d_dirw0 = nullptr;
    std::vector<int32_t> dir_job;    // P
    int device = 0;
    // workspace, allocated with the plan and sized for every batch (max_slots)
    void* d_ws = nullptr;
    // kernel modes beta~(K, L) of the pseudo-spectral form, [K][L], FP64, built
    // on the first pseudo-spectral evaluation (small grids only)
    double* d_beta = nullptr;
    size_t ws_bytes = 0;
    int npts() const { int t = 1; for (int a = 0; a < dim; ++a) t *= n; return t; }
    DevPlan dev() const
    {
        DevPlan d;
        d.dim = dim; d.n = n; d.ntilde = ntilde; d.P = P; d.njobs = (int32_t)jobs.size();
        d.npts = npts();
        d.mode = mode;
        d.jobs = d_jobs; d.dirichlet = d_dirichlet; d.aperp = d_aperp; d.w_default = d_w;
        d.dir_job = d_dir_job;
        d.lam0 = d_lam0;
        d.jobw0 = d_jobw0;
        d.lamb0 = d_lamb0;
        d.dirw0 = d_dirw0;
        d.jt_floats = dim == 2 ? jt_table_floats(jobs.data(), (int)jobs.size(), n) : 0;
        return d;
    }
};

// Host plan construction (no device work).  Returns an empty string on success
// or a message describing the invalid argument.
std::string build_host_plan(int dim, int n, double half_width, int ntilde, int farey_order,
                            int num_dirs, const int32_t* dirs, const double* weights, int line_weight,
                            HostPlan& hp);

bool supported_size(int dim, int n);

// Grids the pseudo-spectral evaluation supports (n^{2d} table): 2D n <= 32, 3D n = 8.
bool pseudo_supported(int dim, int n);
// beta~(K, L) = beta(K, L) - beta(L, L), beta(K, L) = sum_p w_p alpha_p(K) alpha'_p(L),
// in FP64 with the weights rounded to FP32 as the device kernels see them.
std::vector<double> build_pseudo_modes(const HostPlan& hp);

// ------------------------------------------------------------- launch API
// Kernel-side launchers (kernels.hip).  All return hipSuccess or an error.
struct LaunchInfo {
    int grid = 0, block = 0;
    size_t lds = 0;
    int slots = 0;    // resident cell slots that need spectral scratch
    int jsplit = 1;   // > 1: each cell's direction loop is spread over jsplit workgroups
    bool jt = false;  // 2D plain mode: per-job multiplier rows in LDS
};

// Launch shape of a kernel family, chosen by the autotuner or fixed by a
// caller: max_grid > 0 caps the number of workgroups (the persistent kernels
// then take more cells per workgroup); grid_div > 1 runs 1/grid_div of the
// occupancy grid; allow_split = false keeps one workgroup per cell even for
// small 3D batches, split picks the direction split (0 automatic, 1 never,
// G >= 2 forced when batch * G workgroups fit); threads = 1 takes the
// alternative 3D workgroup size (two pencils per lane) where there is one.
struct LaunchLimits {
    int max_grid = 0;
    bool allow_split = true;
    int split = 0;
    int grid_div = 1;
    int threads = 0;
    bool allow_jt = true;   // 2D plain evaluation: per-job multiplier tables may be chosen
};
// true where a 3D grid size has an alternative workgroup size (n = 16, 32)
bool has_alt_threads(int dim, int n);

hipError_t launch_prep(const DevPlan& pl, const float* w, DevScratch s, hipStream_t st);
LaunchInfo eval_launch_info(const DevPlan& pl, int batch, int variant, LaunchLimits lim = LaunchLimits());
hipError_t launch_eval(const DevPlan& pl, int batch, const float* f, float* q, float dt,
                       DevScratch s, const LaunchInfo& li, int variant, hipStream_t st);
LaunchInfo vjp_launch_info(const DevPlan& pl, int batch, int variant, LaunchLimits lim = LaunchLimits());
// Bilinear Q(g, f) (kernels_3d.hip and kernels_2d.hip): multipliers into
// s.lam (Lambda of the unpaired directions) and s.jobw (P direction weights).
hipError_t launch_prep_bilinear(const DevPlan& pl, const float* w, DevScratch s, hipStream_t st);
LaunchInfo bilinear_launch_info(const DevPlan& pl, int batch, int variant, LaunchLimits lim = LaunchLimits());
hipError_t launch_eval_bilinear(const DevPlan& pl, int batch, const float* g, const float* f, float* q, float dt,
                                DevScratch s, const LaunchInfo& li, int variant, hipStream_t st);
hipError_t bil2d_info(const DevPlan& pl, int batch, int variant, LaunchInfo& li, const LaunchLimits& lim);
hipError_t launch_bil2d(const DevPlan& pl, int batch, const float* g, const float* f, float* q, float dt,
                        DevScratch s, const LaunchInfo& li, int variant, hipStream_t st);
// Largest number of resident cell slots any batch can use with the kernels of
// op (0: evaluation, 1: adjoint, 2: bilinear evaluation) and variant, direction-split launches
// included: it bounds the spectral scratch, the grad_w partial rows and the
// split parts, so a plan's workspace can be sized once for every batch.
int max_slots(const DevPlan& pl, int op, int variant, int threads);
hipError_t launch_vjp(const DevPlan& pl, int batch, const float* f, const float* c, float* grad_f,
                      float* grad_w, const float* w, DevScratch s, const LaunchInfo& li, int variant,
                      hipStream_t st);

// 2D launchers (kernels_2d.hip), called by the dispatch in kernels_3d.hip.
hipError_t eval2d_info(const DevPlan& pl, int batch, int variant, LaunchInfo& li, const LaunchLimits& lim);
hipError_t launch_eval2d(const DevPlan& pl, int batch, const float* f, float* q, float dt, DevScratch s,
                         const LaunchInfo& li, int variant, hipStream_t st);
hipError_t vjp2d_info(const DevPlan& pl, int batch, int variant, LaunchInfo& li, const LaunchLimits& lim);
hipError_t launch_vjp2d(const DevPlan& pl, int batch, const float* f, const float* c, float* grad_f,
                        DevScratch s, const LaunchInfo& li, int variant, hipStream_t st);

// ------------------------------------------------------------- heterogeneous batch
enum BatchClass : int32_t { BC_2D8 = 0, BC_2D16 = 1, BC_2D32 = 2, BC_2D64 = 3, BC_3D24 = 4, BC_3D32 = 5,
                            kNumClasses = 6 };
// block-size families of the batched launch: 256 threads (2D n = 8, 16, 32),
// 576 (3D n = 24), 512 (2D n = 64, 3D n = 32)
enum BatchFamily : int32_t { BF_256 = 0, BF_576 = 1, BF_512 = 2, kNumFamilies = 3 };

struct BatchItem {
    int32_t cls, plan, first, count;   // class, plan slot, first entry in cell_off, cells
};

struct BatchDev {
    const BatchItem* items;    // grouped by class, each group ordered by decreasing cost
    int32_t nitems;
    int32_t cls_first[kNumClasses], cls_count[kNumClasses];   // item range of each class
    int32_t cls_static[kNumClasses];   // 1: the class's items cost the same, tickets are assigned statically
    const DevPlan* plans;
    const int64_t* cell_off;   // element offset of each cell, in item order
    int32_t* counter;          // [kNumClasses] work-queue tickets, one queue per class
    float2* spec;              // [grid][slot_elems]
    int64_t slot_elems;
    int64_t gslot;             // near-equilibrium plans: the spectrum of g at slot + gslot and a staging
                               // area at slot + 2 gslot (slot_elems = 3 gslot); else 0
    int64_t fslot;             // 2D plans with more than kFlushJobs jobs: the compensated gain sums
                               // (a float pair per point) at slot + fslot; else 0
    uint32_t fbytes;           // extent of f and q in bytes
    int32_t dtab_floats;       // LDS floats reserved for the Dirichlet tables (D and D - 1 rows)
};

// dtab_floats must be even (the reduction area after the LDS buffers holds doubles)
hipError_t batched_launch_info(int family, int nitems, bool split, LaunchInfo& li, size_t dtab_floats);
size_t batched_slot_elems(int family);
// ------------------------------------------------------------- adaptive direction count
// Cells of one class, each evaluated with the plan of its level: level l when
// the cell's distance from its Maxwellian exceeds l of the increasing
// thresholds (few directions near equilibrium).  The classifier fills one
// queue of cell offsets per level; the persistent launch drains them.
constexpr int kMaxLevels = 8;
struct AdaptDev {
    BatchDev b;                // plans: one per level; cell_off = queue; gslot != 0 when some level
                               // plan is a near-equilibrium plan; items, counter unused
    const int64_t* cell_in;    // [ncells] element offset of each cell, caller's order
    int64_t* queue;            // [nlevels][ncells] offsets of the cells of each level
    int32_t* count;            // [kMaxLevels] cells per level
    int32_t* level;            // [ncells] level of each cell (may be null)
    float* dist;               // [ncells] distance of each cell from its Maxwellian (may be null)
    const float* thr;          // [nlevels - 1] thresholds, increasing
    int32_t nlevels, ncells, cls, cpi;
};
hipError_t adaptive_launch_info(int cls, int ncells, bool split, LaunchInfo& li, size_t dtab_floats);
hipError_t launch_adaptive(const AdaptDev& a, const LaunchInfo& li, const float* f, float* q, float dt,
                           hipStream_t st);

// true if some class of the launch takes dynamic tickets (then a counter reset kernel runs first)
bool batch_uses_counter(const BatchDev& b);
hipError_t launch_batched(int family, const BatchDev& b, const LaunchInfo& li, const float* f, float* q, float dt,
                          hipStream_t st);

// f[c] <- (f[c] + f1[c]) / 2 over the cells (offset, count) of a batch
hipError_t launch_average_cells(const int64_t* off, const int32_t* cnt, int ncells, float* f, const float* f1,
                                hipStream_t st);

// Evaluation of qdvm_eval with its scratch in the caller's device buffer
// (ws, ws_bytes) instead of the plan's workspace (capi.cpp).
qdvm_status eval_with_scratch(qdvm_plan_s* p, int32_t batch, const float* f, float* q, const float* w, float dt,
                              hipStream_t stream, void* ws, size_t ws_bytes);
// Sets the calling thread's last-error text and returns st.
qdvm_status record_error(qdvm_status st, const char* msg);

// Pseudo-spectral evaluation (pseudo.hip): q = Q(f, f) from the FP64 table beta~.
hipError_t launch_pseudo(int dim, int n, int batch, const double* beta, const float* f, float* q, hipStream_t st);

// Forward 2D transform stage at n = 16 (stage.hip): method 0 register FFT,
// 1 DFT as FP32 matrix-core products; `reps` inverse-forward round trips in
// between; out[cell][K1][K0] = fhat(K0, K1).
hipError_t launch_transform_stage(int method, int batch, int reps, const float* f, float2* out, hipStream_t st);

int num_variants(int dim, int n);
int default_variant(int dim, int n);
int device_cu_count();

}  // namespace qdvm
