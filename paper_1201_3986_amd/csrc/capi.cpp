// C interface of the qdvm library: argument checking, plan lifetime, device
// workspace and launches.  See include/qdvm.h for the contract of each call.
#include "../../include/qdvm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
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
    int variant[2] = {-1, -1};
    std::mutex mu;
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
    hipFree(hp.d_ws);
    hp.d_jobs = nullptr;
    hp.d_dirichlet = nullptr;
    hp.d_aperp = nullptr;
    hp.d_w = nullptr;
    hp.d_dir_job = nullptr;
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

// Workspace layout for one call: lam | jobw | spec | spec2 | acc | gw_part.
struct WsLayout {
    size_t lam, jobw, spec, spec2, acc, gw, total;
};

WsLayout ws_layout(const qdvm::HostPlan& hp, int slots, int batch, bool adjoint)
{
    WsLayout L{};
    const size_t npts = (size_t)hp.npts();
    size_t off = 0;
    L.lam = off; off = align_up(off + sizeof(float) * npts);
    L.jobw = off; off = align_up(off + sizeof(float) * std::max<size_t>(1, hp.jobs.size()));
    L.spec = off; off = align_up(off + sizeof(float2) * npts * slots);
    if (adjoint) {
        L.spec2 = off; off = align_up(off + sizeof(float2) * npts * slots);
        L.acc = off; off = align_up(off + sizeof(float2) * npts * slots);
        L.gw = off; off = align_up(off + sizeof(float) * std::max<size_t>(1, hp.jobs.size()) * batch);
    }
    L.total = off;
    return L;
}

qdvm_status ensure_ws(qdvm::HostPlan& hp, size_t bytes, hipStream_t st)
{
    if (hp.ws_bytes >= bytes) return QDVM_OK;
    if (hp.d_ws) {
        // the previous buffer may still be read by work queued on any stream
        (void)st;
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return from_hip(e, "synchronising before workspace growth");
        hipFree(hp.d_ws);
        hp.d_ws = nullptr;
        hp.ws_bytes = 0;
    }
    size_t want = bytes + bytes / 4;
    hipError_t e = hipMalloc(&hp.d_ws, want);
    if (e != hipSuccess) {
        hp.d_ws = nullptr;
        return from_hip(e, "allocating the plan workspace");
    }
    hp.ws_bytes = want;
    return QDVM_OK;
}

qdvm::DevScratch scratch_of(const qdvm::HostPlan& hp, const WsLayout& L, bool adjoint)
{
    char* b = (char*)hp.d_ws;
    qdvm::DevScratch s{};
    s.lam = (float*)(b + L.lam);
    s.jobw = (float*)(b + L.jobw);
    s.spec = (float2*)(b + L.spec);
    if (adjoint) {
        s.spec2 = (float2*)(b + L.spec2);
        s.acc = (float2*)(b + L.acc);
        s.gw_part = (float*)(b + L.gw);
    }
    return s;
}

int effective_variant(const qdvm_plan_s* p, int op) { return p->variant[op] >= 0 ? p->variant[op] : 0; }

qdvm_status do_eval(qdvm_plan_s* p, int batch, const float* f, float* q, const float* w, float dt,
                    hipStream_t st, int variant)
{
    qdvm::HostPlan& hp = p->hp;
    const qdvm::DevPlan pl = hp.dev();
    qdvm::LaunchInfo li = qdvm::eval_launch_info(pl, batch, variant);
    if (li.grid <= 0) return fail(QDVM_EDEVICE, "could not configure the evaluation kernel");
    WsLayout L = ws_layout(hp, li.slots, batch, false);
    qdvm_status s = ensure_ws(hp, L.total, st);
    if (s != QDVM_OK) return s;
    qdvm::DevScratch sc = scratch_of(hp, L, false);
    hipError_t e = qdvm::launch_prep(pl, w ? w : hp.d_w, sc, st);
    if (e != hipSuccess) return from_hip(e, "launching the multiplier preparation");
    e = qdvm::launch_eval(pl, batch, f, q, dt, sc, li, variant, st);
    if (e != hipSuccess) return from_hip(e, "launching the collision kernel");
    hp.last_stream = st;
    return QDVM_OK;
}

qdvm_status do_vjp(qdvm_plan_s* p, int batch, const float* f, const float* c, const float* w, float* gf,
                   float* gw, hipStream_t st, int variant)
{
    qdvm::HostPlan& hp = p->hp;
    const qdvm::DevPlan pl = hp.dev();
    qdvm::LaunchInfo li = qdvm::vjp_launch_info(pl, batch, variant);
    if (li.grid <= 0) return fail(QDVM_EDEVICE, "could not configure the adjoint kernel");
    WsLayout L = ws_layout(hp, li.slots, batch, true);
    qdvm_status s = ensure_ws(hp, L.total, st);
    if (s != QDVM_OK) return s;
    qdvm::DevScratch sc = scratch_of(hp, L, true);
    hipError_t e = qdvm::launch_prep(pl, w ? w : hp.d_w, sc, st);
    if (e != hipSuccess) return from_hip(e, "launching the multiplier preparation");
    e = qdvm::launch_vjp(pl, batch, f, c, gf, gw, w ? w : hp.d_w, sc, li, variant, st);
    if (e != hipSuccess) return from_hip(e, "launching the adjoint kernel");
    hp.last_stream = st;
    return QDVM_OK;
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
                                    desc->num_dirs, desc->dirs, desc->weights, p->hp);
    } catch (const std::bad_alloc&) {
        delete p;
        return fail(QDVM_ENOMEM, "host allocation failed while building the plan");
    } catch (...) {
        delete p;
        return fail(QDVM_EINVAL, "plan construction failed");
    }
    if (!msg.empty()) {
        delete p;
        return from_plan_msg(msg);
    }
    qdvm::HostPlan& hp = p->hp;
    hipError_t e = hipGetDevice(&hp.device);
    std::vector<float> wf(hp.weights.begin(), hp.weights.end());
    if (e == hipSuccess) e = upload(&hp.d_jobs, hp.jobs);
    if (e == hipSuccess) e = upload(&hp.d_dirichlet, hp.dirichlet);
    if (e == hipSuccess) e = upload(&hp.d_aperp, hp.aperp);
    if (e == hipSuccess) e = upload(&hp.d_w, wf);
    if (e == hipSuccess) e = upload(&hp.d_dir_job, hp.dir_job);
    if (e != hipSuccess) {
        free_device(hp);
        delete p;
        return from_hip(e, "uploading plan tables");
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
                                    desc->num_dirs, desc->dirs, desc->weights, hp);
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
    return do_eval(p, batch, f, q, w, dt, stream, effective_variant(p, 0));
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
    return do_vjp(p, batch, f, cot, w, grad_f, grad_w, stream, effective_variant(p, 1));
}

qdvm_status qdvm_set_variant(qdvm_plan_t p, int32_t op, int32_t variant)
{
    if (!p) return fail(QDVM_EINVAL, "null plan");
    if (op < 0 || op > 1) return fail(QDVM_EINVAL, "op must be 0 (eval) or 1 (vjp)");
    if (variant < -1 || variant >= qdvm::num_variants(p->hp.dim, p->hp.n))
        return fail(QDVM_EINVAL, "variant out of range");
    std::lock_guard<std::mutex> lock(p->mu);
    p->variant[op] = variant;
    return QDVM_OK;
}

qdvm_status qdvm_get_variant(qdvm_plan_t p, int32_t op, int32_t* variant)
{
    if (!p || !variant) return fail(QDVM_EINVAL, "null plan or output");
    if (op < 0 || op > 1) return fail(QDVM_EINVAL, "op must be 0 (eval) or 1 (vjp)");
    *variant = effective_variant(p, op);
    return QDVM_OK;
}

qdvm_status qdvm_autotune(qdvm_plan_t p, int32_t batch, hipStream_t st)
{
    if (!p) return fail(QDVM_EINVAL, "null plan");
    if (batch < 1) return fail(QDVM_EINVAL, "batch must be positive");
    std::lock_guard<std::mutex> lock(p->mu);
    qdvm_status s = check_device(p);
    if (s != QDVM_OK) return s;
    const size_t n = (size_t)batch * p->hp.npts();
    float *f = nullptr, *q = nullptr, *g = nullptr;
    hipError_t e = hipMalloc(&f, sizeof(float) * n);
    if (e == hipSuccess) e = hipMalloc(&q, sizeof(float) * n);
    if (e == hipSuccess) e = hipMalloc(&g, sizeof(float) * n);
    if (e == hipSuccess) e = hipMemsetD32Async((hipDeviceptr_t)f, 0x3f800000u, n, st);
    if (e == hipSuccess) e = hipMemsetD32Async((hipDeviceptr_t)g, 0x3f000000u, n, st);
    hipEvent_t a = nullptr, b = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    const int nv = qdvm::num_variants(p->hp.dim, p->hp.n);
    for (int op = 0; op < 2 && e == hipSuccess && s == QDVM_OK; ++op) {
        float best = 1e30f;
        int best_v = 0;
        for (int v = 0; v < nv && e == hipSuccess && s == QDVM_OK; ++v) {
            float ms = 0.f;
            for (int rep = 0; rep < 4 && s == QDVM_OK; ++rep) {
                if (rep == 1) e = hipEventRecord(a, st);
                s = op == 0 ? do_eval(p, batch, f, q, nullptr, 0.f, st, v)
                            : do_vjp(p, batch, f, g, nullptr, q, nullptr, st, v);
            }
            if (s != QDVM_OK || e != hipSuccess) break;
            e = hipEventRecord(b, st);
            if (e == hipSuccess) e = hipEventSynchronize(b);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
            if (e == hipSuccess && ms < best) {
                best = ms;
                best_v = v;
            }
        }
        p->variant[op] = best_v;
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

int32_t qdvm_abi_version(void) { return QDVM_ABI_VERSION; }

}  // extern "C"
