// C interface of the qdvm library: argument checking, plan lifetime, device
// workspace and launches.  See include/qdvm.h for the contract of each call.
#include "../../include/qdvm.h"

#include <string>

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <unistd.h>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "qdvm_internal.h"

struct qdvm_plan_s {
    qdvm::HostPlan hp;
    // launch shape per operation: 0 evaluation (also the bilinear and
    // allocation-free calls), 1 adjoint; radix -1 = the built-in default
    qdvm_launch_config cfg[2] = {{-1, 0, 0, 1}, {-1, 0, 0, 1}};
    std::mutex mu;
};

struct qdvm_batch_s {
    struct Family {
        int fam = 0;
        std::vector<qdvm::BatchItem> items;
        std::vector<int64_t> cell_off;
        std::vector<qdvm::DevPlan> plans;
        qdvm::BatchItem* d_items = nullptr;
        int64_t* d_cell_off = nullptr;
        qdvm::DevPlan* d_plans = nullptr;
        int32_t* d_counter = nullptr;
        float2* d_spec = nullptr;
        qdvm::LaunchInfo li;
        qdvm::BatchDev dev{};
    };
    std::vector<Family> fams;
    std::vector<int64_t> cell_off;   // per cell, in the caller's order
    std::vector<int32_t> cell_cnt;   // n^d of the cell's plan
    int device = 0;
    int32_t ncells = 0;
    uint32_t fbytes = 0;
    double flops = 0.0;   // algorithmic FLOPs of one evaluation of all cells
    std::mutex mu;
};

struct qdvm_adaptive_s {
    int device = 0;
    int32_t ncells = 0, nlevels = 0;
    int64_t* d_cell_in = nullptr;
    int64_t* d_queue = nullptr;
    int32_t* d_count = nullptr;
    float* d_thr = nullptr;
    qdvm::DevPlan* d_plans = nullptr;
    float2* d_spec = nullptr;
    qdvm::LaunchInfo li;
    qdvm::AdaptDev dev{};
    std::mutex mu;
};

struct qdvm_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // two-stage Runge-Kutta: intermediate state and the cells' (offset, count)
    float* f1 = nullptr;
    int64_t* d_off = nullptr;
    int32_t* d_cnt = nullptr;
};

namespace {

thread_local std::string g_last_error;

qdvm_status fail(qdvm_status st, const std::string& msg)
{
    g_last_error = msg;
    return st;
}

qdvm_status from_hip(hipError_t e, const char* what)
{
    if (e == hipSuccess) return QDVM_OK;
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(e == hipErrorOutOfMemory ? QDVM_ENOMEM : QDVM_EDEVICE, m);
}

qdvm_status from_plan_msg(const std::string& m)
{
    if (m.rfind("unsupported", 0) == 0) return fail(QDVM_EUNSUPPORTED, m);
    return fail(QDVM_EINVAL, m);
}

template <class T>
hipError_t upload(T** dst, const std::vector<T>& src)
{
    *dst = nullptr;
    if (src.empty()) return hipSuccess;
    hipError_t e = hipMalloc((void**)dst, sizeof(T) * src.size());
    if (e != hipSuccess) return e;
    return hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
}

void free_device(qdvm::HostPlan& hp)
{
    hipFree(hp.d_jobs);
    hipFree(hp.d_dirichlet);
    hipFree(hp.d_aperp);
    hipFree(hp.d_w);
    hipFree(hp.d_dir_job);
    hipFree(hp.d_lam0);
    hipFree(hp.d_jobw0);
    hipFree(hp.d_lamb0);
    hipFree(hp.d_dirw0);
    hipFree(hp.d_ws);
    hipFree(hp.d_beta);
    hp.d_beta = nullptr;
    hp.d_jobs = nullptr;
    hp.d_dirichlet = nullptr;
    hp.d_aperp = nullptr;
    hp.d_w = nullptr;
    hp.d_dir_job = nullptr;
    hp.d_lam0 = nullptr;
    hp.d_jobw0 = nullptr;
    hp.d_lamb0 = nullptr;
    hp.d_dirw0 = nullptr;
    hp.d_ws = nullptr;
    hp.ws_bytes = 0;
}

qdvm_status check_device(const qdvm_plan_s* p)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return from_hip(e, "hipGetDevice");
    if (dev != p->hp.device) return fail(QDVM_EINVAL, "plan belongs to another device than the current one");
    return QDVM_OK;
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace layout for one call: lam | jobw | spec | spec2 | acc | gw_part | part.
struct WsLayout {
    size_t lam, jobw, spec, spec2, acc, gw, part, total;
};

// Kinds of launch that draw on the workspace.
enum WsKind { WS_EVAL = 0, WS_ADJOINT = 1, WS_BILINEAR = 2 };

// slots: resident cell slots of the launch; rows: grad_w partial rows;
// part_cells: workgroups of a direction-split launch (0 if none).
WsLayout ws_layout(const qdvm::HostPlan& hp, size_t slots, size_t rows, size_t part_cells, int kind)
{
    WsLayout L{};
    const size_t npts = (size_t)hp.npts();
    const size_t njobs = std::max<size_t>(1, hp.jobs.size());
    const bool adjoint = kind == WS_ADJOINT;
    size_t off = 0;
    L.lam = off; off = align_up(off + sizeof(float) * npts);
    // job weights, or the per-direction weights of the bilinear operator
    L.jobw = off; off = align_up(off + sizeof(float) * std::max<size_t>(njobs, (size_t)hp.P));
    L.spec = off; off = align_up(off + sizeof(float2) * npts * slots);
    const bool flush = kind == WS_EVAL && hp.dim == 2 && hp.jobs.size() > (size_t)qdvm::kFlushJobs;
    if (adjoint || kind == WS_BILINEAR || hp.mode || flush) {
        // adjoint: R; bilinear: the transform of g; near-equilibrium evaluation: g and a staging set;
        // 2D evaluation with many jobs: the compensated gain sums
        L.spec2 = off; off = align_up(off + sizeof(float2) * npts * slots * (kind == WS_EVAL ? 2 : 1));
    }
    if (adjoint) {
        L.acc = off; off = align_up(off + sizeof(float2) * npts * slots);
        L.gw = off; off = align_up(off + sizeof(double) * njobs * rows);
    }
    if (part_cells) {
        L.part = off; off = align_up(off + sizeof(float) * npts * part_cells);
    }
    L.total = off;
    return L;
}

WsLayout call_layout(const qdvm::HostPlan& hp, const qdvm::LaunchInfo& li, int batch, int kind)
{
    const size_t slots = (size_t)li.slots;
    return ws_layout(hp, slots, std::min<size_t>((size_t)batch, slots), li.jsplit > 1 ? (size_t)li.grid : 0,
                     kind);
}

// Workspace that serves every batch size, variant and operation of a plan:
// the layout at the largest number of resident slots any launch can use.
qdvm_status workspace_bound(const qdvm::HostPlan& hp, size_t& bytes)
{
    const qdvm::DevPlan pl = hp.dev();
    bytes = 0;
    const int nthreads = qdvm::has_alt_threads(hp.dim, hp.n) ? 2 : 1;
    for (int op = 0; op < 3; ++op)
        for (int v = 0; v < qdvm::num_variants(hp.dim, hp.n); ++v)
            for (int t = 0; t < nthreads; ++t) {
                const int slots = qdvm::max_slots(pl, op, v, t);
                if (slots <= 0)
                    return fail(QDVM_EDEVICE, "could not size the plan workspace (occupancy query failed)");
                const WsLayout L = ws_layout(hp, (size_t)slots, (size_t)slots,
                                             (hp.dim == 3 && op != 2) ? (size_t)slots : 0, op);
                bytes = std::max(bytes, L.total);
            }
    return QDVM_OK;
}

qdvm::DevScratch scratch_of(void* base, const qdvm::HostPlan& hp, const WsLayout& L, int kind, int jsplit)
{
    const bool adjoint = kind == WS_ADJOINT;
    char* b = (char*)base;
    qdvm::DevScratch s{};
    s.lam = (float*)(b + L.lam);
    s.jobw = (float*)(b + L.jobw);
    s.spec = (float2*)(b + L.spec);
    if (L.spec2) s.spec2 = (float2*)(b + L.spec2);   // laid out only where a launch uses it
    if (adjoint) {
        s.acc = (float2*)(b + L.acc);
        s.gw_part = (double*)(b + L.gw);
    }
    if (jsplit > 1) s.part = (float*)(b + L.part);
    return s;
}

// Kernel variant (radix order) and launch shape of an operation.
struct Shape {
    int variant;
    qdvm::LaunchLimits lim;
};

Shape shape_of(const qdvm::HostPlan& hp, const qdvm_launch_config& c)
{
    Shape sh;
    sh.variant = c.radix >= 0 ? c.radix : qdvm::default_variant(hp.dim, hp.n);
    sh.lim.threads = c.threads;
    sh.lim.split = c.split;
    sh.lim.grid_div = c.grid_div;
    return sh;
}

Shape effective_shape(const qdvm_plan_s* p, int op) { return shape_of(p->hp, p->cfg[op]); }

qdvm_status check_config(const qdvm::HostPlan& hp, const qdvm_launch_config& c)
{
    if (c.radix < -1 || c.radix >= qdvm::num_variants(hp.dim, hp.n)) return fail(QDVM_EINVAL, "radix out of range");
    if (c.threads < 0 || c.threads > 1 || (c.threads == 1 && !qdvm::has_alt_threads(hp.dim, hp.n)))
        return fail(QDVM_EINVAL, "threads must be 0, or 1 where an alternative workgroup size exists (3D n = 16, 32)");
    if (c.split < 0 || c.split > 8 || (c.split > 1 && hp.dim != 3))
        return fail(QDVM_EINVAL, "split must be 0 (automatic), 1 (never) or 2..8 (3D only)");
    if (c.grid_div != 1 && c.grid_div != 2 && c.grid_div != 4) return fail(QDVM_EINVAL, "grid_div must be 1, 2 or 4");
    return QDVM_OK;
}

qdvm_status do_eval(qdvm_plan_s* p, int batch, const float* f, float* q, const float* w, float dt,
                    hipStream_t st, const Shape& sh)
{
    qdvm::HostPlan& hp = p->hp;
    const qdvm::DevPlan pl = hp.dev();
    const int variant = sh.variant;
    qdvm::LaunchInfo li = qdvm::eval_launch_info(pl, batch, variant, sh.lim);
    if (li.grid <= 0) return fail(QDVM_EDEVICE, "could not configure the evaluation kernel");
    const WsLayout L = call_layout(hp, li, batch, WS_EVAL);
    if (L.total > hp.ws_bytes) return fail(QDVM_EDEVICE, "internal: launch needs more than the plan workspace");
    qdvm::DevScratch sc = scratch_of(hp.d_ws, hp, L, WS_EVAL, li.jsplit);
    hipError_t e = hipSuccess;
    if (w) {
        e = qdvm::launch_prep(pl, w, sc, st);
        if (e != hipSuccess) return from_hip(e, "launching the multiplier preparation");
    } else {
        sc.lam = hp.d_lam0;
        sc.jobw = hp.d_jobw0;
    }
    e = qdvm::launch_eval(pl, batch, f, q, dt, sc, li, variant, st);
    if (e != hipSuccess) return from_hip(e, "launching the collision kernel");
    return QDVM_OK;
}

qdvm_status do_vjp(qdvm_plan_s* p, int batch, const float* f, const float* c, const float* w, float* gf,
                   float* gw, hipStream_t st, const Shape& sh)
{
    qdvm::HostPlan& hp = p->hp;
    const qdvm::DevPlan pl = hp.dev();
    const int variant = sh.variant;
    qdvm::LaunchInfo li = qdvm::vjp_launch_info(pl, batch, variant, sh.lim);
    if (li.grid <= 0) return fail(QDVM_EDEVICE, "could not configure the adjoint kernel");
    const WsLayout L = call_layout(hp, li, batch, WS_ADJOINT);
    if (L.total > hp.ws_bytes) return fail(QDVM_EDEVICE, "internal: launch needs more than the plan workspace");
    qdvm::DevScratch sc = scratch_of(hp.d_ws, hp, L, WS_ADJOINT, li.jsplit);
    hipError_t e = hipSuccess;
    if (w) {
        e = qdvm::launch_prep(pl, w, sc, st);
        if (e != hipSuccess) return from_hip(e, "launching the multiplier preparation");
    } else {
        sc.lam = hp.d_lam0;
        sc.jobw = hp.d_jobw0;
    }
    e = qdvm::launch_vjp(pl, batch, f, c, gf, gw, w ? w : hp.d_w, sc, li, variant, st);
    if (e != hipSuccess) return from_hip(e, "launching the adjoint kernel");
    return QDVM_OK;
}


qdvm_status do_eval_bilinear(qdvm_plan_s* p, int batch, const float* g, const float* f, float* q, const float* w,
                             float dt, hipStream_t st, const Shape& sh)
{
    qdvm::HostPlan& hp = p->hp;
    const qdvm::DevPlan pl = hp.dev();
    const int variant = sh.variant;
    qdvm::LaunchInfo li = qdvm::bilinear_launch_info(pl, batch, variant, sh.lim);
    if (li.grid <= 0) return fail(QDVM_EDEVICE, "could not configure the bilinear kernel");
    const WsLayout L = call_layout(hp, li, batch, WS_BILINEAR);
    if (L.total > hp.ws_bytes) return fail(QDVM_EDEVICE, "internal: launch needs more than the plan workspace");
    qdvm::DevScratch sc = scratch_of(hp.d_ws, hp, L, WS_BILINEAR, li.jsplit);
    hipError_t e = hipSuccess;
    if (w) {
        e = qdvm::launch_prep_bilinear(pl, w, sc, st);
        if (e != hipSuccess) return from_hip(e, "launching the multiplier preparation");
    } else {
        sc.lam = hp.d_lamb0;
        sc.jobw = hp.d_dirw0;
    }
    e = qdvm::launch_eval_bilinear(pl, batch, g, f, q, dt, sc, li, variant, st);
    if (e != hipSuccess) return from_hip(e, "launching the bilinear kernel");
    return QDVM_OK;
}

// Evaluation whose scratch lives in the given buffer (ws, ws_bytes) instead of
// the plan's workspace: one workgroup per cell (no direction split) and, if the
// resident slots of the natural launch do not fit, fewer workgroups, each
// persistent over more cells.
qdvm_status eval_in(qdvm_plan_s* p, int batch, const float* f, float* q, const float* w, float dt, hipStream_t st,
                    const Shape& sh, void* ws, size_t ws_bytes)
{
    qdvm::HostPlan& hp = p->hp;
    const qdvm::DevPlan pl = hp.dev();
    const int variant = sh.variant;
    qdvm::LaunchLimits lim = sh.lim;
    lim.allow_split = false;
    qdvm::LaunchInfo li = qdvm::eval_launch_info(pl, batch, variant, lim);
    if (li.grid <= 0) return fail(QDVM_EDEVICE, "could not configure the evaluation kernel");
    WsLayout L = call_layout(hp, li, batch, WS_EVAL);
    while (L.total > ws_bytes && li.grid > 1) {
        int g = (int)((double)li.grid * (double)ws_bytes / (double)L.total);
        lim.max_grid = std::max(1, std::min(g, li.grid - 1));
        li = qdvm::eval_launch_info(pl, batch, variant, lim);
        if (li.grid <= 0) return fail(QDVM_EDEVICE, "could not configure the evaluation kernel");
        L = call_layout(hp, li, batch, WS_EVAL);
    }
    if (L.total > ws_bytes) {
        char m[160];
        std::snprintf(m, sizeof m, "one resident cell of this plan needs %zu bytes of scratch, more than the %zu available",
                      L.total, ws_bytes);
        return fail(QDVM_EINVAL, m);
    }
    qdvm::DevScratch sc = scratch_of(ws, hp, L, WS_EVAL, li.jsplit);
    hipError_t e = hipSuccess;
    if (w) {
        e = qdvm::launch_prep(pl, w, sc, st);
        if (e != hipSuccess) return from_hip(e, "launching the multiplier preparation");
    } else {
        sc.lam = hp.d_lam0;
        sc.jobw = hp.d_jobw0;
    }
    e = qdvm::launch_eval(pl, batch, f, q, dt, sc, li, variant, st);
    if (e != hipSuccess) return from_hip(e, "launching the collision kernel");
    return QDVM_OK;
}

int batch_class(int dim, int n)
{
    if (dim == 2) {
        switch (n) {
            case 8: return qdvm::BC_2D8;
            case 16: return qdvm::BC_2D16;
            case 32: return qdvm::BC_2D32;
            case 64: return qdvm::BC_2D64;
        }
    } else if (dim == 3) {
        if (n == 24) return qdvm::BC_3D24;
        if (n == 32) return qdvm::BC_3D32;
    }
    return -1;
}

int class_family(int c)
{
    if (c == qdvm::BC_2D64 || c == qdvm::BC_3D32) return qdvm::BF_512;
    return c == qdvm::BC_3D24 ? qdvm::BF_576 : qdvm::BF_256;
}

int class_cells_per_item(int c)
{
    switch (c) {
        case qdvm::BC_2D8: return 256 / 8;
        case qdvm::BC_2D16: return 256 / 16;
        case qdvm::BC_2D32: return 256 / 32;
        case qdvm::BC_2D64: return 512 / 64;
        default: return 1;
    }
}

double cell_flops(const qdvm::HostPlan& hp)
{
    const double npts = hp.npts();
    const double jobs = (double)hp.jobs.size();
    if (hp.mode == QDVM_MODE_NEAR_EQUILIBRIUM)   // transforms of f and g, two per job, two losses
        return (2 * jobs + 4) * 5.0 * npts * std::log2(npts) + 18.0 * jobs * npts + 16.0 * npts;
    return (jobs + 1) * 5.0 * npts * std::log2(npts) + 9.0 * jobs * npts + 8.0 * npts;
}

void free_batch(qdvm_batch_s* b)
{
    for (auto& F : b->fams) {
        hipFree(F.d_items);
        hipFree(F.d_cell_off);
        hipFree(F.d_plans);
        hipFree(F.d_counter);
        hipFree(F.d_spec);
    }
    b->fams.clear();
}

}  // namespace

extern "C" {

qdvm_status qdvm_plan(const qdvm_desc* desc, qdvm_plan_t* out)
{
    g_last_error.clear();
    if (!desc || !out) return fail(QDVM_EINVAL, "null descriptor or output pointer");
    qdvm_plan_s* p = new (std::nothrow) qdvm_plan_s();
    if (!p) return fail(QDVM_ENOMEM, "host allocation failed");
    std::string msg;
    try {
        msg = qdvm::build_host_plan(desc->dim, desc->n, desc->half_width, desc->ntilde, desc->farey_order,
                                    desc->num_dirs, desc->dirs, desc->weights, desc->line_weight, p->hp);
    } catch (const std::bad_alloc&) {
        delete p;
        return fail(QDVM_ENOMEM, "host allocation failed while building the plan");
    } catch (...) {
        delete p;
        return fail(QDVM_EINVAL, "plan construction failed");
    }
    if (msg.empty() && desc->mode != QDVM_MODE_FULL && desc->mode != QDVM_MODE_NEAR_EQUILIBRIUM)
        msg = "invalid: mode must be QDVM_MODE_FULL (0) or QDVM_MODE_NEAR_EQUILIBRIUM (1)";
    if (!msg.empty()) {
        delete p;
        return from_plan_msg(msg);
    }
    qdvm::HostPlan& hp = p->hp;
    hp.mode = desc->mode;
    hipError_t e = hipGetDevice(&hp.device);
    std::vector<float> wf(hp.weights.begin(), hp.weights.end());
    if (e == hipSuccess) e = upload(&hp.d_jobs, hp.jobs);
    if (e == hipSuccess) e = upload(&hp.d_dirichlet, hp.dirichlet);
    if (e == hipSuccess) e = upload(&hp.d_aperp, hp.aperp);
    if (e == hipSuccess) e = upload(&hp.d_w, wf);
    if (e == hipSuccess) e = upload(&hp.d_dir_job, hp.dir_job);
    // Lambda and the job weights for the plan's own weights, computed once
    if (e == hipSuccess) e = hipMalloc(&hp.d_lam0, sizeof(float) * hp.npts());
    if (e == hipSuccess) e = hipMalloc(&hp.d_jobw0, sizeof(float) * std::max<size_t>(1, hp.jobs.size()));
    if (e == hipSuccess) e = hipMalloc(&hp.d_lamb0, sizeof(float) * hp.npts());
    if (e == hipSuccess) e = hipMalloc(&hp.d_dirw0, sizeof(float) * std::max<size_t>(1, (size_t)hp.P));
    if (e == hipSuccess) {
        qdvm::DevScratch sc{};
        sc.lam = hp.d_lam0;
        sc.jobw = hp.d_jobw0;
        e = qdvm::launch_prep(hp.dev(), hp.d_w, sc, nullptr);
        sc.lam = hp.d_lamb0;
        sc.jobw = hp.d_dirw0;
        if (e == hipSuccess) e = qdvm::launch_prep_bilinear(hp.dev(), hp.d_w, sc, nullptr);
        if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    }
    if (e != hipSuccess) {
        free_device(hp);
        delete p;
        return from_hip(e, "uploading plan tables");
    }
    // the workspace of every later call, sized once for any batch
    size_t ws = 0;
    qdvm_status wst = workspace_bound(hp, ws);
    if (wst == QDVM_OK) {
        e = hipMalloc(&hp.d_ws, ws);
        if (e == hipSuccess)
            hp.ws_bytes = ws;
        else
            wst = from_hip(e, "allocating the plan workspace");
    }
    if (wst != QDVM_OK) {
        free_device(hp);
        delete p;
        return wst;
    }
    *out = p;
    return QDVM_OK;
}

qdvm_status qdvm_describe(const qdvm_desc* desc, int32_t* num_dirs, int32_t* dirs_out, double* weights_out,
                          int32_t* line_len_out, int32_t cap)
{
    g_last_error.clear();
    if (!desc || !num_dirs) return fail(QDVM_EINVAL, "null descriptor or num_dirs pointer");
    if (cap < 0) return fail(QDVM_EINVAL, "negative capacity");
    qdvm::HostPlan hp;
    std::string msg;
    try {
        msg = qdvm::build_host_plan(desc->dim, desc->n, desc->half_width, desc->ntilde, desc->farey_order,
                                    desc->num_dirs, desc->dirs, desc->weights, desc->line_weight, hp);
    } catch (const std::bad_alloc&) {
        return fail(QDVM_ENOMEM, "host allocation failed while building the plan");
    } catch (...) {
        return fail(QDVM_EINVAL, "plan construction failed");
    }
    if (!msg.empty()) return from_plan_msg(msg);
    *num_dirs = hp.P;
    const int m = std::min(cap, hp.P);
    if (dirs_out) std::memcpy(dirs_out, hp.dirs.data(), sizeof(int32_t) * (size_t)m * hp.dim);
    if (weights_out) std::memcpy(weights_out, hp.weights.data(), sizeof(double) * (size_t)m);
    if (line_len_out) std::memcpy(line_len_out, hp.M.data(), sizeof(int32_t) * (size_t)m);
    return QDVM_OK;
}

qdvm_status qdvm_plan_destroy(qdvm_plan_t p)
{
    if (!p) return QDVM_OK;
    qdvm_status st = QDVM_OK;
    if (p->hp.d_ws) {
        // work queued on any stream may still read the plan's memory
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) st = from_hip(e, "synchronising before destroying the plan");
    }
    free_device(p->hp);
    delete p;
    return st;
}

qdvm_status qdvm_plan_info(qdvm_plan_t p, qdvm_plan_info_t* info)
{
    if (!p || !info) return fail(QDVM_EINVAL, "null plan or info pointer");
    info->dim = p->hp.dim;
    info->n = p->hp.n;
    info->ntilde = p->hp.ntilde;
    info->num_dirs = p->hp.P;
    info->num_jobs = (int32_t)p->hp.jobs.size();
    info->h = p->hp.h;
    info->mode = p->hp.mode;
    info->line_weight = p->hp.line_weight;
    return QDVM_OK;
}

qdvm_status qdvm_plan_dirs(qdvm_plan_t p, int32_t* dirs_out, double* weights_out, int32_t* line_len_out)
{
    if (!p) return fail(QDVM_EINVAL, "null plan");
    if (dirs_out) std::memcpy(dirs_out, p->hp.dirs.data(), sizeof(int32_t) * p->hp.dirs.size());
    if (weights_out) std::memcpy(weights_out, p->hp.weights.data(), sizeof(double) * p->hp.weights.size());
    if (line_len_out) std::memcpy(line_len_out, p->hp.M.data(), sizeof(int32_t) * p->hp.M.size());
    return QDVM_OK;
}

qdvm_status qdvm_eval(qdvm_plan_t p, int32_t batch, const float* f, float* q, const float* w, float dt,
                      hipStream_t stream)
{
    if (!p) return fail(QDVM_EINVAL, "null plan");
    if (batch < 0) return fail(QDVM_EINVAL, "negative batch");
    if (batch == 0) return QDVM_OK;
    if (!f || !q) return fail(QDVM_EINVAL, "null f or q");
    if (!std::isfinite(dt)) return fail(QDVM_EINVAL, "dt must be finite");
    std::lock_guard<std::mutex> lock(p->mu);
    qdvm_status s = check_device(p);
    if (s != QDVM_OK) return s;
    return do_eval(p, batch, f, q, w, dt, stream, effective_shape(p, 0));
}

}  // extern "C"

namespace qdvm {

qdvm_status eval_with_scratch(qdvm_plan_t p, int32_t batch, const float* f, float* q, const float* w, float dt,
                              hipStream_t stream, void* ws, size_t ws_bytes)
{
    if (!p) return fail(QDVM_EINVAL, "null plan");
    if (batch < 0) return fail(QDVM_EINVAL, "negative batch");
    if (batch == 0) return QDVM_OK;
    if (!f || !q) return fail(QDVM_EINVAL, "null f or q");
    if (!std::isfinite(dt)) return fail(QDVM_EINVAL, "dt must be finite");
    std::lock_guard<std::mutex> lock(p->mu);
    qdvm_status s = check_device(p);
    if (s != QDVM_OK) return s;
    return eval_in(p, batch, f, q, w, dt, stream, effective_shape(p, 0), ws, ws_bytes);
}

qdvm_status record_error(qdvm_status st, const char* msg) { return fail(st, msg); }

}  // namespace qdvm

extern "C" {

qdvm_status qdvm_eval_bilinear(qdvm_plan_t p, int32_t batch, const float* g, const float* f, float* q,
                               const float* w, float dt, hipStream_t stream)
{
    if (!p) return fail(QDVM_EINVAL, "null plan");
    if (batch < 0) return fail(QDVM_EINVAL, "negative batch");
    if (batch == 0) return QDVM_OK;
    if (!g || !f || !q) return fail(QDVM_EINVAL, "null g, f or q");
    if (!std::isfinite(dt)) return fail(QDVM_EINVAL, "dt must be finite");
    std::lock_guard<std::mutex> lock(p->mu);
    qdvm_status s = check_device(p);
    if (s != QDVM_OK) return s;
    return do_eval_bilinear(p, batch, g, f, q, w, dt, stream, effective_shape(p, 0));
}

qdvm_status qdvm_vjp(qdvm_plan_t p, int32_t batch, const float* f, const float* cot, const float* w,
                     float* grad_f, float* grad_w, hipStream_t stream)
{
    if (!p) return fail(QDVM_EINVAL, "null plan");
    if (batch < 0) return fail(QDVM_EINVAL, "negative batch");
    if (batch == 0) return QDVM_OK;
    if (!f || !cot || !grad_f) return fail(QDVM_EINVAL, "null f, cot or grad_f");
    if (grad_f == f || grad_f == cot) return fail(QDVM_EINVAL, "grad_f must not alias f or cot");
    std::lock_guard<std::mutex> lock(p->mu);
    qdvm_status s = check_device(p);
    if (s != QDVM_OK) return s;
    return do_vjp(p, batch, f, cot, w, grad_f, grad_w, stream, effective_shape(p, 1));
}

qdvm_status qdvm_set_variant(qdvm_plan_t p, int32_t op, int32_t variant)
{
    if (!p) return fail(QDVM_EINVAL, "null plan");
    if (op < 0 || op > 1) return fail(QDVM_EINVAL, "op must be 0 (eval) or 1 (vjp)");
    if (variant < -1 || variant >= qdvm::num_variants(p->hp.dim, p->hp.n))
        return fail(QDVM_EINVAL, "variant out of range");
    std::lock_guard<std::mutex> lock(p->mu);
    p->cfg[op].radix = variant;
    return QDVM_OK;
}

qdvm_status qdvm_get_variant(qdvm_plan_t p, int32_t op, int32_t* variant)
{
    if (!p || !variant) return fail(QDVM_EINVAL, "null plan or output");
    if (op < 0 || op > 1) return fail(QDVM_EINVAL, "op must be 0 (eval) or 1 (vjp)");
    *variant = effective_shape(p, op).variant;
    return QDVM_OK;
}

qdvm_status qdvm_set_config(qdvm_plan_t p, int32_t op, const qdvm_launch_config* cfg)
{
    if (!p) return fail(QDVM_EINVAL, "null plan");
    if (op < 0 || op > 1) return fail(QDVM_EINVAL, "op must be 0 (eval) or 1 (vjp)");
    const qdvm_launch_config def = {-1, 0, 0, 1};
    const qdvm_launch_config c = cfg ? *cfg : def;
    const qdvm_status s = check_config(p->hp, c);
    if (s != QDVM_OK) return s;
    std::lock_guard<std::mutex> lock(p->mu);
    p->cfg[op] = c;
    return QDVM_OK;
}

qdvm_status qdvm_get_config(qdvm_plan_t p, int32_t op, qdvm_launch_config* cfg)
{
    if (!p || !cfg) return fail(QDVM_EINVAL, "null plan or output");
    if (op < 0 || op > 1) return fail(QDVM_EINVAL, "op must be 0 (eval) or 1 (vjp)");
    std::lock_guard<std::mutex> lock(p->mu);
    *cfg = p->cfg[op];
    if (cfg->radix < 0) cfg->radix = qdvm::default_variant(p->hp.dim, p->hp.n);
    return QDVM_OK;
}

namespace {

// ---------------------------------------------------------------- tuning cache
// One line per tuned (device, plan shape, operation, batch class):
//   <key> <radix> <threads> <split> <grid_div> <ms>
// key = qdvm4:<arch>:<cus>:<d>:<n>:<Nt>:<P>:<jobs>:<mode>:<line_weight>:<op>:<ceil log2 batch>.

std::string tune_key(const qdvm::HostPlan& hp, int op, int batch)
{
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    int cus = 0;
    if (hipGetDeviceProperties(&prop, hp.device) == hipSuccess) {
        arch = prop.gcnArchName;
        cus = prop.multiProcessorCount;
    }
    for (char& ch : arch)
        if (ch == ' ' || ch == ':') ch = '_';
    int bclass = 0;
    while ((1 << bclass) < batch && bclass < 30) ++bclass;
    char buf[256];
    std::snprintf(buf, sizeof buf, "qdvm4:%s:%d:%d:%d:%d:%d:%d:%d:%d:%d:%d", arch.c_str(), cus, hp.dim, hp.n,
                  hp.ntilde, hp.P, (int)hp.jobs.size(), hp.mode, hp.line_weight, op, bclass);
    return buf;
}

bool cache_lookup(const char* path, const std::string& key, qdvm_launch_config& out)
{
    FILE* fh = std::fopen(path, "r");
    if (!fh) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, fh)) {
        char k[300];
        qdvm_launch_config c{};
        float ms = 0.f;
        if (std::sscanf(line, "%299s %d %d %d %d %f", k, &c.radix, &c.threads, &c.split, &c.grid_div, &ms) == 6 &&
            key == k) {
            out = c;
            found = true;   // the last entry of a key wins
        }
    }
    std::fclose(fh);
    return found;
}

// Replaces or appends the entry of `key`; the file is rewritten through a
// temporary and renamed, so a concurrent reader never sees a partial file.
void cache_store(const char* path, const std::string& key, const qdvm_launch_config& c, float ms)
{
    std::vector<std::string> lines;
    if (FILE* fh = std::fopen(path, "r")) {
        char line[512];
        while (std::fgets(line, sizeof line, fh)) {
            char k[300];
            if (std::sscanf(line, "%299s", k) == 1 && key == k) continue;
            lines.push_back(line);
        }
        std::fclose(fh);
    }
    char entry[512];
    std::snprintf(entry, sizeof entry, "%s %d %d %d %d %.5f\n", key.c_str(), c.radix, c.threads, c.split, c.grid_div,
                  ms);
    lines.push_back(entry);
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long)::getpid());
    FILE* out = std::fopen(tmp.c_str(), "w");
    if (!out) return;
    for (const auto& l : lines) std::fputs(l.c_str(), out);
    std::fclose(out);
    std::rename(tmp.c_str(), path);
}

}  // namespace

qdvm_status qdvm_autotune(qdvm_plan_t p, int32_t batch, hipStream_t st)
{
    if (!p) return fail(QDVM_EINVAL, "null plan");
    if (batch < 1) return fail(QDVM_EINVAL, "batch must be positive");
    std::lock_guard<std::mutex> lock(p->mu);
    qdvm_status s = check_device(p);
    if (s != QDVM_OK) return s;
    qdvm::HostPlan& hp = p->hp;
    const char* cache = std::getenv("QDVM_TUNE_CACHE");
    if (cache && *cache) {
        qdvm_launch_config c0{}, c1{};
        if (cache_lookup(cache, tune_key(hp, 0, batch), c0) && cache_lookup(cache, tune_key(hp, 1, batch), c1) &&
            check_config(hp, c0) == QDVM_OK && check_config(hp, c1) == QDVM_OK) {
            p->cfg[0] = c0;
            p->cfg[1] = c1;
            return QDVM_OK;
        }
    }
    const size_t n = (size_t)batch * hp.npts();
    float *f = nullptr, *q = nullptr, *g = nullptr;
    hipError_t e = hipMalloc(&f, sizeof(float) * n);
    if (e == hipSuccess) e = hipMalloc(&q, sizeof(float) * n);
    if (e == hipSuccess) e = hipMalloc(&g, sizeof(float) * n);
    if (e == hipSuccess) e = hipMemsetD32Async((hipDeviceptr_t)f, 0x3f800000u, n, st);
    if (e == hipSuccess) e = hipMemsetD32Async((hipDeviceptr_t)g, 0x3f000000u, n, st);
    hipEvent_t a = nullptr, b = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    const qdvm::DevPlan pl = hp.dev();
    const int nv = qdvm::num_variants(hp.dim, hp.n);
    const int nthreads = qdvm::has_alt_threads(hp.dim, hp.n) ? 2 : 1;
    const int splits3[] = {0, 1, 2, 4, 8};
    for (int op = 0; op < 2 && e == hipSuccess && s == QDVM_OK; ++op) {
        float best = 1e30f;
        qdvm_launch_config best_c = {-1, 0, 0, 1};
        std::vector<std::vector<int>> seen;   // launches already timed: (variant, grid, block, jsplit)
        const int nsplit = hp.dim == 3 ? 5 : 1;
        for (int v = 0; v < nv; ++v)
            for (int t = 0; t < nthreads; ++t)
                for (int gd : {1, 2})
                    for (int si = 0; si < nsplit && e == hipSuccess && s == QDVM_OK; ++si) {
                        const qdvm_launch_config c = {v, t, splits3[si], gd};
                        const Shape sh = shape_of(hp, c);
                        const qdvm::LaunchInfo li = op == 0 ? qdvm::eval_launch_info(pl, batch, v, sh.lim)
                                                            : qdvm::vjp_launch_info(pl, batch, v, sh.lim);
                        if (li.grid <= 0) continue;
                        const std::vector<int> sig = {v, li.grid, li.block, li.jsplit};
                        if (std::find(seen.begin(), seen.end(), sig) != seen.end()) continue;
                        seen.push_back(sig);
                        float ms = 0.f;
                        for (int rep = 0; rep < 4 && s == QDVM_OK; ++rep) {
                            if (rep == 1) e = hipEventRecord(a, st);
                            s = op == 0 ? do_eval(p, batch, f, q, nullptr, 0.f, st, sh)
                                        : do_vjp(p, batch, f, g, nullptr, q, nullptr, st, sh);
                        }
                        if (s != QDVM_OK || e != hipSuccess) break;
                        e = hipEventRecord(b, st);
                        if (e == hipSuccess) e = hipEventSynchronize(b);
                        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
                        if (e == hipSuccess && ms < best) {
                            best = ms;
                            best_c = c;
                        }
                    }
        if (s == QDVM_OK && e == hipSuccess) {
            p->cfg[op] = best_c;
            if (cache && *cache) cache_store(cache, tune_key(hp, op, batch), best_c, best / 3.f);
        }
    }
    if (a) hipEventDestroy(a);
    if (b) hipEventDestroy(b);
    hipStreamSynchronize(st);
    hipFree(f);
    hipFree(q);
    hipFree(g);
    if (s != QDVM_OK) return s;
    return from_hip(e, "autotuning");
}

qdvm_status qdvm_batch_plan(int32_t ncells, const qdvm_plan_t* cell_plan, const int64_t* cell_offset,
                            qdvm_batch_t* out)
{
    g_last_error.clear();
    if (!out) return fail(QDVM_EINVAL, "null output pointer");
    if (ncells < 0) return fail(QDVM_EINVAL, "negative ncells");
    if (ncells > 0 && (!cell_plan || !cell_offset)) return fail(QDVM_EINVAL, "null cell_plan or cell_offset");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return from_hip(e, "hipGetDevice");
    int64_t max_end = 0;
    double flops = 0.0;
    for (int32_t c = 0; c < ncells; ++c) {
        const qdvm_plan_s* p = cell_plan[c];
        if (!p) return fail(QDVM_EINVAL, "null plan for cell " + std::to_string(c));
        if (p->hp.device != dev) return fail(QDVM_EINVAL, "a plan belongs to another device than the current one");
        if (batch_class(p->hp.dim, p->hp.n) < 0)
            return fail(QDVM_EUNSUPPORTED, "batched launch supports 2D n in {8,16,32,64} and 3D n in {24,32}");
        if (cell_offset[c] < 0) return fail(QDVM_EINVAL, "negative cell offset");
        max_end = std::max<int64_t>(max_end, cell_offset[c] + p->hp.npts());
        flops += cell_flops(p->hp);
    }
    if (max_end * 4 >= (int64_t(1) << 31)) return fail(QDVM_EINVAL, "f extent must stay below 2 GiB per batch");
    qdvm_batch_s* b = new (std::nothrow) qdvm_batch_s();
    if (!b) return fail(QDVM_ENOMEM, "host allocation failed");
    b->device = dev;
    b->ncells = ncells;
    try {
        b->cell_off.assign(cell_offset, cell_offset + ncells);
        b->cell_cnt.resize(ncells);
        for (int32_t c = 0; c < ncells; ++c) b->cell_cnt[c] = cell_plan[c]->hp.npts();
    } catch (const std::bad_alloc&) {
        delete b;
        return fail(QDVM_ENOMEM, "host allocation failed");
    }
    b->fbytes = (uint32_t)(max_end * 4);
    b->flops = flops;
    for (int fam = 0; fam < qdvm::kNumFamilies; ++fam) {
        // groups of cells with the same (class, plan), in order of first appearance
        std::vector<std::pair<std::pair<int, const qdvm_plan_s*>, std::vector<int32_t>>> groups;
        for (int32_t c = 0; c < ncells; ++c) {
            const qdvm_plan_s* p = cell_plan[c];
            const int cls = batch_class(p->hp.dim, p->hp.n);
            if (class_family(cls) != fam) continue;
            auto key = std::make_pair(cls, p);
            size_t gi = 0;
            while (gi < groups.size() && groups[gi].first != key) ++gi;
            if (gi == groups.size()) groups.push_back({key, {}});
            groups[gi].second.push_back(c);
        }
        if (groups.empty()) continue;
        qdvm_batch_s::Family F;
        F.fam = fam;
        std::vector<const qdvm_plan_s*> plan_of_slot;
        struct Tmp {
            qdvm::BatchItem it;
            std::vector<int32_t> cells;
            double cost;
        };
        std::vector<Tmp> tmp;
        size_t dtab_floats = 2;
        bool any_split = false;
        for (auto& g : groups) {
            const int cls = g.first.first;
            const qdvm_plan_s* p = g.first.second;
            int slot = -1;
            for (size_t k = 0; k < plan_of_slot.size(); ++k)
                if (plan_of_slot[k] == p) slot = (int)k;
            if (slot < 0) {
                slot = (int)plan_of_slot.size();
                plan_of_slot.push_back(p);
                F.plans.push_back(p->hp.dev());
                dtab_floats = std::max<size_t>(dtab_floats, (size_t)2 * (p->hp.ntilde + 1) * p->hp.n);
                any_split = any_split || p->hp.mode == QDVM_MODE_NEAR_EQUILIBRIUM;
            }
            const int cpi = class_cells_per_item(cls);
            for (size_t k = 0; k < g.second.size(); k += cpi) {
                Tmp t;
                t.it.cls = cls;
                t.it.plan = slot;
                t.it.count = (int32_t)std::min<size_t>(cpi, g.second.size() - k);
                t.cells.assign(g.second.begin() + k, g.second.begin() + k + t.it.count);
                t.cost = cell_flops(p->hp) * t.it.count;
                tmp.push_back(t);
            }
        }
        // grouped by class (one queue each); within a class the most expensive
        // items first, so that the tail of each queue is made of small ones
        std::stable_sort(tmp.begin(), tmp.end(), [](const Tmp& a, const Tmp& c) {
            return a.it.cls != c.it.cls ? a.it.cls < c.it.cls : a.cost > c.cost;
        });
        for (int k = 0; k < qdvm::kNumClasses; ++k) {
            F.dev.cls_first[k] = F.dev.cls_count[k] = 0;
            F.dev.cls_static[k] = 1;
        }
        double first_cost[qdvm::kNumClasses] = {0, 0, 0, 0, 0, 0};
        for (auto& t : tmp) {
            t.it.first = (int32_t)F.cell_off.size();
            for (int32_t c : t.cells) F.cell_off.push_back(cell_offset[c]);
            if (F.dev.cls_count[t.it.cls]++ == 0) {
                F.dev.cls_first[t.it.cls] = (int32_t)F.items.size();
                first_cost[t.it.cls] = t.cost;
            } else if (t.cost != first_cost[t.it.cls]) {
                F.dev.cls_static[t.it.cls] = 0;   // uneven items: dynamic queue
            }
            F.items.push_back(t.it);
        }
        dtab_floats = (dtab_floats + 1) & ~size_t(1);
        e = qdvm::batched_launch_info(fam, (int)F.items.size(), any_split, F.li, dtab_floats);
        if (e != hipSuccess || F.li.grid <= 0) {
            free_batch(b);
            delete b;
            return from_hip(e == hipSuccess ? hipErrorInvalidValue : e, "configuring the batched kernel");
        }
        const size_t base_slot = qdvm::batched_slot_elems(fam);
        bool any_flush = false;   // 2D plans whose gain sums are flushed (cells_2d.h)
        for (const auto& pp : F.plans) any_flush = any_flush || (pp.dim == 2 && pp.njobs > qdvm::kFlushJobs);
        const size_t fslot = any_split ? 3 * base_slot : base_slot;          // f, g and staging spectra
        const size_t slot_elems = fslot + (any_flush ? base_slot : 0);
        e = hipMalloc(&F.d_items, sizeof(qdvm::BatchItem) * F.items.size());
        if (e == hipSuccess) e = hipMemcpy(F.d_items, F.items.data(), sizeof(qdvm::BatchItem) * F.items.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMalloc(&F.d_cell_off, sizeof(int64_t) * F.cell_off.size());
        if (e == hipSuccess) e = hipMemcpy(F.d_cell_off, F.cell_off.data(), sizeof(int64_t) * F.cell_off.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMalloc(&F.d_plans, sizeof(qdvm::DevPlan) * F.plans.size());
        if (e == hipSuccess) e = hipMemcpy(F.d_plans, F.plans.data(), sizeof(qdvm::DevPlan) * F.plans.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMalloc(&F.d_counter, sizeof(int32_t) * qdvm::kNumClasses);
        if (e == hipSuccess) e = hipMalloc(&F.d_spec, sizeof(float2) * slot_elems * F.li.grid);
        if (e != hipSuccess) {
            b->fams.push_back(F);
            free_batch(b);
            delete b;
            return from_hip(e, "allocating the batch tables");
        }
        F.dev.items = F.d_items;
        F.dev.nitems = (int32_t)F.items.size();
        F.dev.plans = F.d_plans;
        F.dev.cell_off = F.d_cell_off;
        F.dev.counter = F.d_counter;
        F.dev.spec = F.d_spec;
        F.dev.slot_elems = (int64_t)slot_elems;
        F.dev.gslot = any_split ? (int64_t)base_slot : 0;
        F.dev.fslot = any_flush ? (int64_t)fslot : 0;
        F.dev.fbytes = b->fbytes;
        F.dev.dtab_floats = (int32_t)dtab_floats;
        b->fams.push_back(F);
    }
    *out = b;
    return QDVM_OK;
}

qdvm_status qdvm_batch_destroy(qdvm_batch_t b)
{
    if (!b) return QDVM_OK;
    qdvm_status st = QDVM_OK;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) st = from_hip(e, "synchronising before destroying the batch");
    free_batch(b);
    delete b;
    return st;
}

qdvm_status qdvm_batch_info(qdvm_batch_t b, int32_t* launches, int32_t* items, double* flops)
{
    if (!b) return fail(QDVM_EINVAL, "null batch");
    int32_t n = 0;
    for (auto& F : b->fams) n += (int32_t)F.items.size();
    int32_t nl = 0;
    for (auto& F : b->fams) nl += 1 + (qdvm::batch_uses_counter(F.dev) ? 1 : 0);
    if (launches) *launches = nl;
    if (items) *items = n;
    if (flops) *flops = b->flops;
    return QDVM_OK;
}

qdvm_status qdvm_batch_eval(qdvm_batch_t b, const float* f, float* q, float dt, hipStream_t st)
{
    if (!b) return fail(QDVM_EINVAL, "null batch");
    if (b->ncells == 0) return QDVM_OK;
    if (!f || !q) return fail(QDVM_EINVAL, "null f or q");
    if (!std::isfinite(dt)) return fail(QDVM_EINVAL, "dt must be finite");
    std::lock_guard<std::mutex> lock(b->mu);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return from_hip(e, "hipGetDevice");
    if (dev != b->device) return fail(QDVM_EINVAL, "batch belongs to another device than the current one");
    for (auto& F : b->fams) {
        e = qdvm::launch_batched(F.fam, F.dev, F.li, f, q, dt, st);
        if (e != hipSuccess) return from_hip(e, "launching the batched kernel");
    }
    return QDVM_OK;
}

qdvm_status qdvm_eval_batched(int32_t ncells, const qdvm_plan_t* cell_plan, const int64_t* cell_offset,
                              const float* f, float* q, float dt, hipStream_t st)
{
    qdvm_batch_t b = nullptr;
    qdvm_status s = qdvm_batch_plan(ncells, cell_plan, cell_offset, &b);
    if (s != QDVM_OK) return s;
    s = qdvm_batch_eval(b, f, q, dt, st);
    if (s == QDVM_OK) {
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) s = from_hip(e, "synchronising the batched evaluation");
    }
    qdvm_status s2 = qdvm_batch_destroy(b);
    return s != QDVM_OK ? s : s2;
}

namespace {

void free_graph(qdvm_graph_s* g)
{
    if (g->exec) hipGraphExecDestroy(g->exec);
    if (g->graph) hipGraphDestroy(g->graph);
    hipFree(g->f1);
    hipFree(g->d_off);
    hipFree(g->d_cnt);
    delete g;
}

}  // namespace

qdvm_status qdvm_step_graph_create_scheme(qdvm_batch_t b, float* f, float dt, int32_t scheme, hipStream_t st,
                                          qdvm_graph_t* out)
{
    if (!b || !f || !out) return fail(QDVM_EINVAL, "null batch, f or output");
    if (!st) return fail(QDVM_EINVAL, "graph capture needs a non-default stream");
    if (!std::isfinite(dt)) return fail(QDVM_EINVAL, "dt must be finite");
    if (scheme != QDVM_STEP_EULER && scheme != QDVM_STEP_RK2)
        return fail(QDVM_EINVAL, "scheme must be QDVM_STEP_EULER or QDVM_STEP_RK2");
    std::lock_guard<std::mutex> lock(b->mu);
    qdvm_graph_s* g = new (std::nothrow) qdvm_graph_s();
    if (!g) return fail(QDVM_ENOMEM, "host allocation failed");
    hipError_t e = hipSuccess;
    if (scheme == QDVM_STEP_RK2 && b->ncells > 0) {
        e = hipMalloc(&g->f1, std::max<size_t>(b->fbytes, 4));
        if (e == hipSuccess) e = hipMalloc(&g->d_off, sizeof(int64_t) * b->cell_off.size());
        if (e == hipSuccess) e = hipMalloc(&g->d_cnt, sizeof(int32_t) * b->cell_cnt.size());
        if (e == hipSuccess)
            e = hipMemcpy(g->d_off, b->cell_off.data(), sizeof(int64_t) * b->cell_off.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(g->d_cnt, b->cell_cnt.data(), sizeof(int32_t) * b->cell_cnt.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            free_graph(g);
            return from_hip(e, "allocating the Runge-Kutta stage buffer");
        }
    }
    e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        free_graph(g);
        return from_hip(e, "beginning stream capture");
    }
    hipError_t le = hipSuccess;
    if (scheme == QDVM_STEP_EULER) {
        for (auto& F : b->fams) {   // f <- f + dt Q(f)
            le = qdvm::launch_batched(F.fam, F.dev, F.li, f, f, dt, st);
            if (le != hipSuccess) break;
        }
    } else {
        for (auto& F : b->fams) {   // f1 <- f + dt Q(f)
            le = qdvm::launch_batched(F.fam, F.dev, F.li, f, g->f1, dt, st);
            if (le != hipSuccess) break;
        }
        for (auto& F : b->fams) {   // f1 <- f1 + dt Q(f1)
            if (le != hipSuccess) break;
            le = qdvm::launch_batched(F.fam, F.dev, F.li, g->f1, g->f1, dt, st);
        }
        if (le == hipSuccess)       // f <- (f + f1) / 2
            le = qdvm::launch_average_cells(g->d_off, g->d_cnt, b->ncells, f, g->f1, st);
    }
    e = hipStreamEndCapture(st, &g->graph);
    if (le == hipSuccess && e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (le != hipSuccess || e != hipSuccess) {
        free_graph(g);
        return from_hip(le != hipSuccess ? le : e, "capturing the time step");
    }
    *out = g;
    return QDVM_OK;
}

qdvm_status qdvm_step_graph_create(qdvm_batch_t b, float* f, float dt, hipStream_t st, qdvm_graph_t* out)
{
    return qdvm_step_graph_create_scheme(b, f, dt, QDVM_STEP_EULER, st, out);
}

qdvm_status qdvm_step_graph_launch(qdvm_graph_t g, hipStream_t st)
{
    if (!g) return fail(QDVM_EINVAL, "null graph");
    return from_hip(hipGraphLaunch(g->exec, st), "launching the step graph");
}

qdvm_status qdvm_step_graph_destroy(qdvm_graph_t g)
{
    if (!g) return QDVM_OK;
    // a replay may still be running on any stream
    const hipError_t e = hipDeviceSynchronize();
    free_graph(g);
    return from_hip(e, "destroying the step graph");
}

qdvm_status qdvm_eval_pseudo_spectral(qdvm_plan_t p, int32_t batch, const float* f, float* q, hipStream_t stream)
{
    if (!p) return fail(QDVM_EINVAL, "null plan");
    if (batch < 0) return fail(QDVM_EINVAL, "negative batch");
    if (!qdvm::pseudo_supported(p->hp.dim, p->hp.n))
        return fail(QDVM_EUNSUPPORTED, "the pseudo-spectral form is built for 2D n <= 32 and 3D n = 8");
    if (batch == 0) return QDVM_OK;
    if (!f || !q) return fail(QDVM_EINVAL, "null f or q");
    if (f == q) return fail(QDVM_EINVAL, "q must not alias f");
    std::lock_guard<std::mutex> lock(p->mu);
    qdvm_status s = check_device(p);
    if (s != QDVM_OK) return s;
    qdvm::HostPlan& hp = p->hp;
    if (!hp.d_beta) {
        std::vector<double> beta;
        try {
            beta = qdvm::build_pseudo_modes(hp);
        } catch (const std::bad_alloc&) {
            return fail(QDVM_ENOMEM, "host allocation failed while building the kernel modes");
        }
        double* d = nullptr;
        hipError_t e = upload(&d, beta);
        if (e != hipSuccess) {
            hipFree(d);
            return from_hip(e, "uploading the kernel modes");
        }
        hp.d_beta = d;
    }
    return from_hip(qdvm::launch_pseudo(hp.dim, hp.n, batch, hp.d_beta, f, q, stream),
                    "launching the pseudo-spectral kernel");
}

qdvm_status qdvm_transform_stage(int32_t method, int32_t dim, int32_t n, int32_t batch, int32_t reps,
                                 const float* f, float* fhat, hipStream_t stream)
{
    if (method != 0 && method != 1) return fail(QDVM_EINVAL, "method must be 0 (register FFT) or 1 (matrix-core DFT)");
    if (reps < 0 || reps > 64) return fail(QDVM_EINVAL, "reps must be in [0, 64]");
    if (batch < 0) return fail(QDVM_EINVAL, "negative batch");
    if (dim != 2 || n != 16) return fail(QDVM_EUNSUPPORTED, "the transform stage is built for 2D n = 16 only");
    if (batch == 0) return QDVM_OK;
    if (!f || !fhat) return fail(QDVM_EINVAL, "null f or fhat");
    return from_hip(qdvm::launch_transform_stage(method, batch, reps, f, (float2*)fhat, stream),
                    "launching the transform stage");
}

const char* qdvm_status_string(qdvm_status s)
{
    switch (s) {
        case QDVM_OK: return "ok";
        case QDVM_EINVAL: return "invalid argument";
        case QDVM_EUNSUPPORTED: return "unsupported";
        case QDVM_ENOMEM: return "out of device memory";
        case QDVM_EDEVICE: return "device error";
    }
    return "unknown status";
}

const char* qdvm_last_error(void) { return g_last_error.c_str(); }

namespace {

void free_adaptive(qdvm_adaptive_s* a)
{
    if (a->d_cell_in) (void)hipFree(a->d_cell_in);
    if (a->d_queue) (void)hipFree(a->d_queue);
    if (a->d_count) (void)hipFree(a->d_count);
    if (a->d_thr) (void)hipFree(a->d_thr);
    if (a->d_plans) (void)hipFree(a->d_plans);
    if (a->d_spec) (void)hipFree(a->d_spec);
}

}  // namespace

qdvm_status qdvm_adaptive_plan(int32_t ncells, const int64_t* cell_offset, int32_t nlevels,
                               const qdvm_plan_t* level_plan, const float* threshold, qdvm_adaptive_t* out)
{
    g_last_error.clear();
    if (!out) return fail(QDVM_EINVAL, "null output pointer");
    if (ncells < 1) return fail(QDVM_EINVAL, "ncells must be positive");
    if (!cell_offset || !level_plan) return fail(QDVM_EINVAL, "null cell_offset or level_plan");
    if (nlevels < 1 || nlevels > qdvm::kMaxLevels) return fail(QDVM_EINVAL, "nlevels must be in 1..8");
    if (nlevels > 1 && !threshold) return fail(QDVM_EINVAL, "null threshold");
    for (int32_t l = 0; l + 1 < nlevels; ++l) {
        if (!std::isfinite(threshold[l])) return fail(QDVM_EINVAL, "thresholds must be finite");
        if (l > 0 && !(threshold[l] > threshold[l - 1]))
            return fail(QDVM_EINVAL, "thresholds must be strictly increasing");
    }
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return from_hip(e, "hipGetDevice");
    size_t dtab_floats = 0;
    bool any_split = false;
    for (int32_t l = 0; l < nlevels; ++l) {
        const qdvm_plan_s* p = level_plan[l];
        if (!p) return fail(QDVM_EINVAL, "null plan for level " + std::to_string(l));
        if (p->hp.device != dev) return fail(QDVM_EINVAL, "a plan belongs to another device than the current one");
        if (p->hp.dim != level_plan[0]->hp.dim || p->hp.n != level_plan[0]->hp.n)
            return fail(QDVM_EINVAL, "the level plans must share dim and n");
        any_split = any_split || p->hp.mode == QDVM_MODE_NEAR_EQUILIBRIUM;
        dtab_floats = std::max<size_t>(dtab_floats, (size_t)2 * (p->hp.ntilde + 1) * p->hp.n);
    }
    const int cls = batch_class(level_plan[0]->hp.dim, level_plan[0]->hp.n);
    if (cls < 0) return fail(QDVM_EUNSUPPORTED, "adaptive batches support 2D n in {8,16,32,64} and 3D n in {24,32}");
    const int64_t npts = level_plan[0]->hp.npts();
    int64_t max_end = 0;
    for (int32_t c = 0; c < ncells; ++c) {
        if (cell_offset[c] < 0) return fail(QDVM_EINVAL, "negative cell offset");
        max_end = std::max<int64_t>(max_end, cell_offset[c] + npts);
    }
    if (max_end * 4 >= (int64_t(1) << 31)) return fail(QDVM_EINVAL, "f extent must stay below 2 GiB per batch");
    qdvm_adaptive_s* a = new (std::nothrow) qdvm_adaptive_s();
    if (!a) return fail(QDVM_ENOMEM, "host allocation failed");
    a->device = dev;
    a->ncells = ncells;
    a->nlevels = nlevels;
    dtab_floats = (dtab_floats + 1) & ~size_t(1);
    e = qdvm::adaptive_launch_info(cls, ncells, any_split, a->li, dtab_floats);
    if (e != hipSuccess || a->li.grid <= 0) {
        delete a;
        return from_hip(e == hipSuccess ? hipErrorInvalidValue : e, "configuring the adaptive kernel");
    }
    std::vector<qdvm::DevPlan> plans;
    for (int32_t l = 0; l < nlevels; ++l) plans.push_back(level_plan[l]->hp.dev());
    const size_t base_slot = qdvm::batched_slot_elems(class_family(cls));
    bool any_flush = false;   // 2D plans whose gain sums are flushed (cells_2d.h)
    for (const auto& pp : plans) any_flush = any_flush || (pp.dim == 2 && pp.njobs > qdvm::kFlushJobs);
    const size_t fslot = any_split ? 3 * base_slot : base_slot;   // f, g and staging spectra
    const size_t slot_elems = fslot + (any_flush ? base_slot : 0);
    e = hipMalloc(&a->d_cell_in, sizeof(int64_t) * ncells);
    if (e == hipSuccess) e = hipMemcpy(a->d_cell_in, cell_offset, sizeof(int64_t) * ncells, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&a->d_queue, sizeof(int64_t) * (size_t)nlevels * ncells);
    if (e == hipSuccess) e = hipMalloc(&a->d_count, sizeof(int32_t) * qdvm::kMaxLevels);
    if (e == hipSuccess) e = hipMalloc(&a->d_thr, sizeof(float) * qdvm::kMaxLevels);
    if (e == hipSuccess && nlevels > 1)
        e = hipMemcpy(a->d_thr, threshold, sizeof(float) * (nlevels - 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&a->d_plans, sizeof(qdvm::DevPlan) * nlevels);
    if (e == hipSuccess) e = hipMemcpy(a->d_plans, plans.data(), sizeof(qdvm::DevPlan) * nlevels, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&a->d_spec, sizeof(float2) * slot_elems * a->li.grid);
    if (e != hipSuccess) {
        free_adaptive(a);
        delete a;
        return from_hip(e, "allocating the adaptive batch tables");
    }
    qdvm::AdaptDev& d = a->dev;
    d.b.plans = a->d_plans;
    d.b.cell_off = a->d_queue;
    d.b.spec = a->d_spec;
    d.b.slot_elems = (int64_t)slot_elems;
    d.b.gslot = any_split ? (int64_t)base_slot : 0;
    d.b.fslot = any_flush ? (int64_t)fslot : 0;
    d.b.fbytes = (uint32_t)(max_end * 4);
    d.b.dtab_floats = (int32_t)dtab_floats;
    d.cell_in = a->d_cell_in;
    d.queue = a->d_queue;
    d.count = a->d_count;
    d.thr = a->d_thr;
    d.nlevels = nlevels;
    d.ncells = ncells;
    d.cls = cls;
    d.cpi = class_cells_per_item(cls);
    *out = a;
    return QDVM_OK;
}

qdvm_status qdvm_adaptive_eval(qdvm_adaptive_t a, const float* f, float* q, float dt, int32_t* level, float* dist,
                               hipStream_t st)
{
    if (!a) return fail(QDVM_EINVAL, "null adaptive batch");
    if (!f || !q) return fail(QDVM_EINVAL, "null f or q");
    if (!std::isfinite(dt)) return fail(QDVM_EINVAL, "dt must be finite");
    std::lock_guard<std::mutex> lock(a->mu);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return from_hip(e, "hipGetDevice");
    if (dev != a->device) return fail(QDVM_EINVAL, "adaptive batch belongs to another device than the current one");
    qdvm::AdaptDev d = a->dev;
    d.level = level;
    d.dist = dist;
    e = qdvm::launch_adaptive(d, a->li, f, q, dt, st);
    if (e != hipSuccess) return from_hip(e, "launching the adaptive kernels");
    return QDVM_OK;
}

qdvm_status qdvm_adaptive_destroy(qdvm_adaptive_t a)
{
    if (!a) return QDVM_OK;
    qdvm_status st = QDVM_OK;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) st = from_hip(e, "synchronising before destroying the adaptive batch");
    free_adaptive(a);
    delete a;
    return st;
}

int32_t qdvm_abi_version(void) { return QDVM_ABI_VERSION; }

}  // extern "C"
