/*
 * qdvm.h -- C interface of the MI355X (gfx950) implementation of the fast
 * discrete-velocity (DVM) Boltzmann collision operator of
 *   C. Mouhot, L. Pareschi, T. Rey, "Convolutive decomposition and fast
 *   summation methods for discrete-velocity approximations of the Boltzmann
 *   equation".
 *
 * The operator (Sec. 2.3, eq. (2.9), restricted by the direction decomposition
 * of Sec. 3.2, eqs. (3.6)-(3.7), with the decoupled weights a(k) b(l) of
 * eq. (3.3), b = 1 and a constant on each lattice line):
 *
 *   Q_i = sum_p w_p sum_{0<|m|<=M_p} sum_{l.e_p=0, |l|_inf<=Nt}
 *              [ f(i + m e_p) f(i + l) - f(i) f(i + m e_p + l) ],
 *   M_p = floor(Nt / |e_p|_inf),
 *
 * on the periodic grid (Z/nZ)^d with n points per axis.  It is evaluated by
 * FFT convolutions (Sec. 3.3) at O(P n^d log n) cost.
 *
 * Conventions common to every call
 *   - A cell is one distribution function f on the n^d grid, FP32, C order
 *     (last axis fastest), point j at velocity v_j = -R + j h, h = 2R/n.
 *     The grid origin does not enter Q; only moments need the velocities.
 *   - Array arguments named "device" are device pointers owned by the caller;
 *     "host" arguments are host pointers read during the call only.
 *   - Launches are asynchronous on the given HIP stream (NULL = the legacy
 *     default stream).  Errors detected on the host are returned at once and
 *     nothing is launched or written; faults inside kernels surface as
 *     QDVM_EDEVICE from a later synchronising call.
 *   - A plan's device workspace is allocated with the plan, sized for every
 *     batch size, and shared by all calls on that plan: qdvm_eval and qdvm_vjp
 *     never allocate, free or synchronise (they may be captured into a HIP
 *     graph), and calls on one plan must be ordered (one stream, or externally
 *     serialised).  Different plans are independent.  Plans are bound to the
 *     device that was current at creation; calls must be made with that
 *     device current.
 *   - No exception crosses this interface.
 */
#ifndef QDVM_H
#define QDVM_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QDVM_ABI_VERSION 4

typedef enum {
    QDVM_OK = 0,
    QDVM_EINVAL = -1,        /* invalid argument (null pointer, bad size, bad direction...) */
    QDVM_EUNSUPPORTED = -2,  /* a valid request outside the compiled set (grid size) */
    QDVM_ENOMEM = -3,        /* device allocation failed */
    QDVM_EDEVICE = -4        /* HIP runtime or kernel failure */
} qdvm_status;

typedef struct qdvm_plan_s* qdvm_plan_t;   /* opaque, immutable after creation */
typedef struct qdvm_batch_s* qdvm_batch_t; /* opaque heterogeneous batch (cells of several plans) */
typedef struct qdvm_graph_s* qdvm_graph_t; /* opaque captured Euler step */
typedef struct qdvm_adaptive_s* qdvm_adaptive_t; /* opaque adaptive-direction-count batch */

/*
 * Plan descriptor: the parameters of Sec. 3.3 (n, the truncation Nt through
 * the box, the direction set through Nbar) and the weights of Sec. 3.2.
 */
typedef struct {
    int32_t dim;            /* d in {2, 3} */
    int32_t n;              /* points per axis; supported: 2D {8,16,32,64}, 3D {8,16,24,32} */
    double half_width;      /* R > 0: the grid spans [-R, R)^d, h = 2R/n */
    int32_t ntilde;         /* Nt; 0 selects floor(n / (3 + sqrt 2)) (Sec. 4).  Requires
                               1 <= Nt and 2 Nt + 1 <= n */
    int32_t farey_order;    /* Nbar >= 1: use every line of [-Nbar, Nbar]^d (Sec. 3.2, the set
                               A^{d-1}); used when dirs == NULL and num_dirs == 0 */
    int32_t num_dirs;       /* P > 0 with dirs == NULL: the first P lines in canonical order
                               (|e|_inf, then |e|_2^2, then components ascending) */
    const int32_t* dirs;    /* optional host array P x d: primitive vectors, first nonzero
                               component positive, no two on the same line */
    const double* weights;  /* optional host array of P weights w_p; NULL selects the profile's
                               default (below) */
    int32_t mode;           /* QDVM_MODE_FULL or QDVM_MODE_NEAR_EQUILIBRIUM (below) */
    int32_t line_weight;    /* weight a(k) of the points k = m e_p of a line (below) */
} qdvm_desc;

/*
 * Line-weight profiles: the factor a(k) of the decoupled kernel a(k) b(l),
 * b = 1 (Sec. 3.2, eq. (3.3)), at the points k = m e_p, 0 < |m| <= M_p.
 *   QDVM_LINE_UNIFORM: a(m e_p) = w_p, the paper's lattice weights
 *     a(k) = h^(2d-1) |k| / gcd(k) = h^(2d-1) |e_p|_2 (Sec. 3.2, after
 *     eq. (3.3)) by default.  2D perpendicular lines share a transform.
 *   QDVM_LINE_DELTA: a(m e_p) = w_p / |m| with default w_p = h^(2d-2), i.e.
 *     a(k) = h^(2d-2) / gcd(k): the lattice quadrature of delta(x . y) in the
 *     Carleman form of Sec. 2.2 for a constant kernel (a point of the line or
 *     plane orthogonal to k stands for a length or area h^(d-1) |k| / gcd(k),
 *     divided by |x| = h |k|).  With it the 2D Maxwell-molecule operator
 *     converges to the BKW solution of Sec. 4 as n grows; the uniform
 *     profile's operator does not (its continuum limit carries an extra
 *     factor |x|).  No 2D pairing (the pair's terms differ when the weight
 *     varies along a line), so P transforms per cell in 2D.
 */
#define QDVM_LINE_UNIFORM 0
#define QDVM_LINE_DELTA 1

/*
 * Evaluation modes.
 *   QDVM_MODE_FULL: Q(f, f) of Sec. 3.2 in FP32 arithmetic; the rounding error
 *     scales with |f|^2, so near equilibrium (where Q is small against |f|^2)
 *     the relative error grows.
 *   QDVM_MODE_NEAR_EQUILIBRIUM: per cell, M is the discrete Maxwellian with the
 *     mass, mean and temperature of f on the index grid (computed in FP64),
 *     g = f - M, and the result is Q(f, f) - Q(M, M) = Q(g, f) + Q(M, g),
 *     evaluated with no transform mixing f-sized and g-sized data, so the error
 *     scales with |f| |g|.  Q(M, M) vanishes for an unwrapped discrete
 *     Maxwellian (every pair of the discrete sum of Sec. 2.3 cancels); what is left
 *     out is its periodic-wrap residue.  About twice the transforms of
 *     QDVM_MODE_FULL.  A cell whose moments do not define a Maxwellian (mass
 *     <= 0, or index-space temperature <= 1/4) takes M = 0, i.e. Q(f, f).
 *     qdvm_vjp ignores the mode and differentiates Q(f, f).
 */
#define QDVM_MODE_FULL 0
#define QDVM_MODE_NEAR_EQUILIBRIUM 1

typedef struct {
    int32_t dim, n, ntilde;
    int32_t num_dirs;       /* P */
    int32_t num_jobs;       /* inverse transforms per cell in the direction loop */
    double h;
    int32_t mode;           /* the descriptor's evaluation mode */
    int32_t line_weight;    /* the descriptor's line-weight profile */
} qdvm_plan_info_t;

/* Build a plan: direction set, line lengths M_p, weights and FP64-built
 * multiplier tables, uploaded to the current device, and the workspace of
 * every later evaluation and adjoint call (spectral scratch for the resident
 * cells of the largest launch; tens to a few hundred MiB depending on the
 * grid).  Synchronises the device.  *out is written only on success.
 * EINVAL for an invalid descriptor, EUNSUPPORTED for n outside the supported
 * set, ENOMEM/EDEVICE for device failures. */
qdvm_status qdvm_plan(const qdvm_desc* desc, qdvm_plan_t* out);

/* Destroy a plan.  Synchronises the device (work on any stream may still read
 * the plan), then frees its device memory.  NULL is accepted (no-op). */
qdvm_status qdvm_plan_destroy(qdvm_plan_t plan);

/* Host-only preview of the direction set a descriptor selects (no device
 * work): *num_dirs receives P; up to `cap` lines are written to dirs_out
 * (host, cap x d int32), weights_out (host, cap doubles) and line_len_out
 * (host, cap int32: M_p); any output may be NULL.  Same validation as
 * qdvm_plan. */
qdvm_status qdvm_describe(const qdvm_desc* desc, int32_t* num_dirs, int32_t* dirs_out, double* weights_out,
                          int32_t* line_len_out, int32_t cap);

/* Plan parameters (host struct written on success). */
qdvm_status qdvm_plan_info(qdvm_plan_t plan, qdvm_plan_info_t* info);

/* Direction set of a plan: dirs_out (host, P x d int32), weights_out (host,
 * P doubles: the default or descriptor weights), line_len_out (host, P int32:
 * M_p).  Any output may be NULL. */
qdvm_status qdvm_plan_dirs(qdvm_plan_t plan, int32_t* dirs_out, double* weights_out, int32_t* line_len_out);

/*
 * Evaluate Q(f, f) for `batch` cells that share the plan.
 *   f  device, batch * n^d floats, cells back to back.
 *   q  device, batch * n^d floats: q = Q(f) when dt == 0, else the forward
 *      Euler update q = f + dt Q(f) (Prop. 3.3, eq. (3.8)).  q may equal f
 *      (in place); partial overlap is not allowed.
 *   w  optional device array of P FP32 weights overriding the plan's for
 *      this call only (the plan is never modified); NULL uses the plan's.
 * batch == 0 is a no-op.  Inputs with NaN/Inf propagate into the output.
 */
qdvm_status qdvm_eval(qdvm_plan_t plan, int32_t batch, const float* f, float* q, const float* w,
                      float dt, hipStream_t stream);

/*
 * The bilinear operator Q(g, f) for `batch` cells sharing the plan (the
 * consistency statement of Sec. 2.3 is written for D(g, f); Q(f, f) is its
 * diagonal):
 *   Q(g, f)_i = sum_p w_p sum_{0<|m|<=M_p} sum_{l.e_p=0, |l|_inf<=Nt}
 *                 [ g(i + m e_p) f(i + l) - g(i) f(i + m e_p + l) ],
 * i.e. the gain takes g along the line and f over the plane, the loss is
 * g(i) times the collision frequency of f.
 *   g, f  device, batch * n^d floats each, cells back to back.
 *   q     device, batch * n^d floats: q = Q(g, f) when dt == 0, else the
 *         forward Euler update of the first argument, q = g + dt Q(g, f)
 *         (the evolution of g in the field of f).  q may equal g or f;
 *         partial overlap is not allowed.
 *   w     optional device array of P FP32 weights, as in qdvm_eval.
 * The plan's evaluation mode is ignored (always the plain FP32 form), and
 * the kernel variant is the evaluation's (op 0).  Each direction costs one
 * inverse transform (2D perpendicular pairs do not share one here: Q(g, f) is
 * not symmetric under exchanging the two lines), plus two forward transforms
 * and one loss transform per cell.  Never allocates or synchronises.
 */
qdvm_status qdvm_eval_bilinear(qdvm_plan_t plan, int32_t batch, const float* g, const float* f, float* q,
                               const float* w, float dt, hipStream_t stream);

/*
 * qdvm_eval for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments and results, but the scratch of the launch is a static
 * device array of this library (qdvm_noalloc_scratch_bytes(): 32 MiB per GPU,
 * held until the process ends) instead of the plan's workspace.  The call
 * allocates, frees and synchronises nothing; if the natural launch's resident
 * cells do not fit in the array it runs fewer, persistent workgroups (never
 * a direction-split launch), so results equal qdvm_eval's up to summation
 * order (bit for bit in 2D).  EINVAL if one resident cell of the plan needs
 * more scratch than the array holds.  Every call on one GPU uses that GPU's
 * one array: calls that overlap in time on one GPU (concurrent streams or
 * threads) race and must be serialised by the caller.  The plan itself is
 * created beforehand (qdvm_plan allocates).
 */
qdvm_status qdvm_eval_noalloc(qdvm_plan_t plan, int32_t batch, const float* f, float* q, const float* w,
                              float dt, hipStream_t stream);
size_t qdvm_noalloc_scratch_bytes(void);

/*
 * Vector-Jacobian product of Q with respect to f and the weights, for `batch`
 * cells sharing the plan, with cotangent `cot`:
 *   grad_f  device, batch * n^d floats, overwritten: d<cot, Q>/df per cell.
 *           Must not overlap f or cot.
 *   grad_w  optional device array of P floats, overwritten: d<cot, Q>/dw_p
 *           summed over the batch in a fixed order (deterministic).  A
 *           direction with M_p = 0 gets 0.
 *   w       optional device weights as in qdvm_eval.
 */
qdvm_status qdvm_vjp(qdvm_plan_t plan, int32_t batch, const float* f, const float* cot, const float* w,
                     float* grad_f, float* grad_w, hipStream_t stream);

/*
 * Heterogeneous batch: many spatial cells, each with its own plan (grid size,
 * direction set, weights), evaluated in one persistent launch per block-size
 * family present (256 threads: 2D n = 8, 16, 32; 576: 3D n = 24; 512: 2D
 * n = 64 and 3D n = 32), with a device work queue ordered by cost.  Sec. 3.3
 * notes that the direction set may vary with position; each cell is the
 * single-cell operator of its plan.
 *   cell_plan    host array of ncells plans (the same plan may repeat); every
 *                plan on the current device.  3D n = 8 and 16 are not
 *                supported here (EUNSUPPORTED).
 *   cell_offset  host array of ncells element offsets of each cell in f/q;
 *                cells must not overlap and the largest offset + n^d must stay
 *                below 2^29 elements (2 GiB).
 * The batch holds its work list, plan table, queue counter and scratch on
 * the device; the plans must outlive it.  Calls on one batch must be ordered.
 */
qdvm_status qdvm_batch_plan(int32_t ncells, const qdvm_plan_t* cell_plan, const int64_t* cell_offset,
                            qdvm_batch_t* out);
qdvm_status qdvm_batch_destroy(qdvm_batch_t batch);   /* synchronises the device first; NULL is a no-op */
/* launches (kernel launches per evaluation: one per block-size family, plus a
 * queue-counter reset before a family whose items differ in cost), work
 * items, algorithmic FLOPs of one evaluation;
 * each output may be NULL */
qdvm_status qdvm_batch_info(qdvm_batch_t batch, int32_t* launches, int32_t* items, double* flops);
/* q = Q(f) per cell (dt == 0) or q = f + dt Q(f); f and q are device arrays
 * addressed by the batch's cell offsets; q may equal f (in place). */
qdvm_status qdvm_batch_eval(qdvm_batch_t batch, const float* f, float* q, float dt, hipStream_t stream);
/* One-shot form: builds a batch, evaluates, synchronises `stream`, destroys it. */
qdvm_status qdvm_eval_batched(int32_t ncells, const qdvm_plan_t* cell_plan, const int64_t* cell_offset,
                              const float* f, float* q, float dt, hipStream_t stream);

/* Capture one in-place forward-Euler step f <- f + dt Q(f) of a batch (queue
 * reset kernel + persistent launch, no memset nodes) into a HIP graph on a
 * non-default stream; each launch replays it on `stream`.  The graph reuses
 * the batch's device state, so the batch must outlive it and replays must be
 * ordered. */
qdvm_status qdvm_step_graph_create(qdvm_batch_t batch, float* f, float dt, hipStream_t capture_stream,
                                   qdvm_graph_t* out);

/* The same with a choice of scheme:
 *   QDVM_STEP_EULER  f <- f + dt Q(f)                      (as qdvm_step_graph_create)
 *   QDVM_STEP_RK2    the two-stage TVD Runge-Kutta step the paper integrates
 *                    with (Sec. 4): f1 = f + dt Q(f), f <- (f + f1 + dt Q(f1)) / 2.
 *                    Each stage keeps f >= 0 when dt times the loss frequency
 *                    is below 1 (Prop. 3.3) and the average is convex.  The
 *                    graph owns a device buffer of the batch's extent for f1;
 *                    only the cells are written (gaps keep their values).
 * EINVAL for an unknown scheme. */
#define QDVM_STEP_EULER 0
#define QDVM_STEP_RK2 1
qdvm_status qdvm_step_graph_create_scheme(qdvm_batch_t batch, float* f, float dt, int32_t scheme,
                                          hipStream_t capture_stream, qdvm_graph_t* out);
qdvm_status qdvm_step_graph_launch(qdvm_graph_t graph, hipStream_t stream);
qdvm_status qdvm_step_graph_destroy(qdvm_graph_t graph);   /* synchronises the device first; NULL is a no-op */

/*
 * Adaptive direction count (Sec. 3.3, the remark after the complexity count:
 * the number of directions may depend on the position, fewer where the
 * distribution is close to equilibrium).  An adaptive batch evaluates cells of
 * one grid size, each with the plan of its level.  The level of a cell is the
 * number of thresholds exceeded by its distance from equilibrium
 *     r = sum_i |f_i - M_i| / sum_i |f_i|        (r = 0 for a zero cell),
 * M the Maxwellian of the cell's moments on the index grid (mass s0, mean mu,
 * temperature var = (sum |i|^2 f / s0 - |mu|^2) / d, as in the
 * near-equilibrium mode; M = 0 when s0 <= 0 or var <= 1/4), computed in FP64
 * on the device at every evaluation.
 *   cell_offset: host, ncells element offsets (as for qdvm_batch_plan).
 *   level_plan:  host, nlevels (1..8) plans of one dim and n in the batched
 *                set, either mode, on the current device; borrowed (they must
 *                outlive the adaptive batch).  List them by increasing cost
 *                (fewest directions first): the launch drains the last first.
 *   threshold:   host, nlevels - 1 finite, strictly increasing values.
 * The adaptive batch holds its level queues, counters and spectral slots on
 * the device: calls on one adaptive batch must be ordered (one stream, or
 * externally serialised).
 * Errors: EINVAL (null or inconsistent arguments), EUNSUPPORTED (a grid outside
 * the batched set), ENOMEM / EDEVICE.
 */
qdvm_status qdvm_adaptive_plan(int32_t ncells, const int64_t* cell_offset, int32_t nlevels,
                               const qdvm_plan_t* level_plan, const float* threshold, qdvm_adaptive_t* out);
/* q = Q(f) (dt == 0) or f + dt Q(f) per cell with its level's directions; q may
 * equal f.  level (int32) and dist (float) are optional device outputs of
 * ncells entries (each cell's level and r).  Three launches on the stream: a
 * counter reset, the classifier (one workgroup per cell) and the persistent
 * drain of the level queues; nothing is allocated. */
qdvm_status qdvm_adaptive_eval(qdvm_adaptive_t adaptive, const float* f, float* q, float dt, int32_t* level,
                               float* dist, hipStream_t stream);
qdvm_status qdvm_adaptive_destroy(qdvm_adaptive_t adaptive);   /* synchronises the device first; NULL is a no-op */

/*
 * Launch shape of the evaluation (op 0: qdvm_eval, qdvm_eval_bilinear,
 * qdvm_eval_noalloc) and of the adjoint (op 1: qdvm_vjp) of a plan.  Every
 * shape computes the same operator; they differ in speed and, by summation
 * order, in the last bits.
 */
typedef struct {
    int32_t radix;      /* FFT radix order of the pencil transforms, 0 or 1; -1: the built-in default
                           (4 x 8 for 3D n = 32, else 0) */
    int32_t threads;    /* 3D n = 16 and 32: 0 one pencil per lane (256 / 1024 threads per cell),
                           1 two pencils per lane (128 / 512 threads); else 0 */
    int32_t split;      /* 3D: direction split of small batches, 0 automatic (when the batch leaves
                           more than half of the workgroup slots idle), 1 never, G = 2..8 that many
                           workgroups per cell whenever they fit; 2D: 0 or 1 */
    int32_t grid_div;   /* 1, 2 or 4: persistent workgroups = occupancy x CUs / grid_div */
} qdvm_launch_config;

/* Set (cfg NULL: restore the defaults) or read the launch shape of op 0 or 1.
 * EINVAL for a field out of range.  The plan's workspace covers every shape. */
qdvm_status qdvm_set_config(qdvm_plan_t plan, int32_t op, const qdvm_launch_config* cfg);
qdvm_status qdvm_get_config(qdvm_plan_t plan, int32_t op, qdvm_launch_config* cfg);

/* Radix order alone (the `radix` field above): -1 restores the default. */
qdvm_status qdvm_set_variant(qdvm_plan_t plan, int32_t op, int32_t variant);
qdvm_status qdvm_get_variant(qdvm_plan_t plan, int32_t op, int32_t* variant);

/*
 * Autotuner: times every distinct launch of the shape space above (radix x
 * threads x grid_div x split) for evaluation and adjoint on `batch` synthetic
 * cells on `stream` and keeps the fastest per op.  If the environment
 * variable QDVM_TUNE_CACHE names a file, shapes are looked up there first,
 * keyed by (GPU architecture and CU count, d, n, Nt, P, jobs, mode, line
 * weight, op, ceil(log2 batch)), and the tuned ones are written back (the file
 * is replaced through a temporary and a rename; concurrent tuners may lose an
 * entry, never corrupt the file).  Allocates and frees its synthetic buffers
 * and synchronises `stream`.
 */
qdvm_status qdvm_autotune(qdvm_plan_t plan, int32_t batch, hipStream_t stream);

/*
 * Q(f, f) by the pseudo-spectral form of Sec. 3.1: q~_I = sum_{K+L=I}
 * (beta(K, L) - beta(L, L)) f~_K f~_L with the kernel modes of eq. (3.2),
 * beta(K, L) = sum_p w_p alpha_p(K) alpha'_p(L) under the plan's direction
 * set, weights and line-weight profile, evaluated by direct O(n^{2d}) sums in
 * FP64 on the device (forward DFT, mode sum, inverse DFT): an independent
 * second evaluation of the plan's operator for small grids, to check the
 * fast FP32 path against on the GPU.  2D n <= 32 and 3D n = 8 (EUNSUPPORTED
 * otherwise).  f, q device, batch * n^d floats; q must not alias f.  The
 * first call on a plan builds its n^{2d} FP64 table of modes on the host,
 * uploads it (allocates) and synchronises; later calls are asynchronous.
 * The plan's mode and the evaluation's launch shape do not apply.
 */
qdvm_status qdvm_eval_pseudo_spectral(qdvm_plan_t plan, int32_t batch, const float* f, float* q,
                                      hipStream_t stream);

/*
 * The forward transform of the 2D evaluation as a stage by itself, for
 * measuring the choice of transform (Sec. 3.1: the operator lives on the DFT
 * of f): fhat[cell][K1][K0] = sum_j f[cell][j0][j1] exp(-2 pi i (K.j) / n),
 * complex FP32 pairs, for `batch` real n x n cells (device pointers, cells
 * back to back).  method 0: the register FFT the collision kernels run;
 * method 1: the DFT as dense products on the FP32 matrix cores (MFMA).
 * reps (0..64): inverse-forward round trips on the spectrum in registers
 * before it is written (each scaled back by 1/n^2, so the result is the same
 * transform up to rounding): with reps > 0 the stage costs 2 reps + 1
 * transforms per cell for one read and one write, as the transforms of the
 * fused evaluation do.  Only dim = 2, n = 16 (EUNSUPPORTED otherwise).  The
 * evaluation itself always uses the FFT (the measured faster of the two).
 */
qdvm_status qdvm_transform_stage(int32_t method, int32_t dim, int32_t n, int32_t batch, int32_t reps,
                                 const float* f, float* fhat, hipStream_t stream);

const char* qdvm_status_string(qdvm_status status);
/* Detail of the last error raised on the calling thread ("" if none). */
const char* qdvm_last_error(void);
int32_t qdvm_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* QDVM_H */
