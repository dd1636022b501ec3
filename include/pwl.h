/*
 * pwl.h - C ABI of the MI355X (gfx950) library for evaluating a continuous
 * function through its near-optimal continuous piecewise-linear (CPWL)
 * approximation.
 *
 * Method: Berjon, Gallego, Cuevas, Moran, Garcia, "Optimal Piecewise Linear
 * Function Approximation for GPU-based Applications", IEEE Trans. Cybernetics
 * 2015 (arXiv 1510.02975).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Point arrays (x, y, g, dx, seg) and the value arrays v_override / dv are
 *    caller-owned DEVICE memory on the current HIP device, contiguous FP32
 *    (int32 for seg).  16-byte alignment of all point arrays selects the
 *    vectorised kernels; any other alignment is accepted and served by a
 *    scalar kernel.
 *  - Tables (pwl_table) and batches (pwl_batch) are opaque, owned by the
 *    library and resident in device memory; free them with the matching
 *    *_free call.
 *  - `stream` is a hipStream_t passed as void*; NULL means the default
 *    stream.  Every call is enqueued on that stream and returns without
 *    waiting, except pwl_table_check, pwl_table_download and the create
 *    calls, which synchronise the stream they are given.
 *  - Arguments are validated on the host before anything is enqueued; an
 *    invalid call enqueues nothing and returns a negative pwl_status.  HIP
 *    runtime failures return PWL_EHIP.  pwl_last_error() then returns a
 *    message (thread-local; valid until the next failing call on the thread).
 *  - n = 0 points is valid and does nothing.
 *
 * Evaluation semantics (Algorithm 1, Sec. IV of the paper, plus the readings
 * this library fixes where the paper is silent):
 *  - x is clamped to the table domain [a, b] (constant extension);
 *  - x = b lies in the last segment with fractional distance 1;
 *  - a point exactly on an interior knot belongs to the segment on its right;
 *  - NaN x gives NaN y and NaN dL/dx and contributes nothing to dL/dv.
 */
#ifndef PWL_H
#define PWL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PWL_ABI_VERSION 2
#define PWL_MAX_N 4096     /* segments per table: the table lives in LDS */
#define PWL_MAX_PARAMS 6

typedef enum pwl_status {
    PWL_OK = 0,
    PWL_EINVAL = -1,     /* invalid argument (nothing was enqueued)          */
    PWL_ENOMEM = -2,     /* device allocation failed                         */
    PWL_EHIP = -3,       /* HIP runtime error (message in pwl_last_error)    */
    PWL_EKNOTS = -4,     /* FP32 knots are not strictly increasing           */
    PWL_ECAPACITY = -5   /* N above PWL_MAX_N or a size limit of the library */
} pwl_status;

/* The approximated functions f (the paper's normalisation constants are
 * folded into amp).  params may be NULL/short; missing ones take the
 * defaults in brackets. */
typedef enum pwl_func {
    PWL_F_GAUSSIAN = 0,    /* amp * exp(-x^2 / (2 s^2));  params {s [1], amp [1]}, s > 0   (Sec. VI-A) */
    PWL_F_LORENTZIAN = 1,  /* amp / (1 + (x / g)^2);      params {g [1], amp [1]}, g > 0   (Sec. VI-B) */
    PWL_F_BESSEL_J0 = 2,   /* amp * J0(x);                params {amp [1]}                 (Sec. VI-C) */
    PWL_F_POLY = 16,       /* c0 + c1 x + ... + c5 x^5;   params {c0 .. c5} (test function)           */
    PWL_F_EXP = 17,        /* amp * exp(alpha x);         params {alpha [1], amp [1]} (test function)  */
    PWL_F_SAMPLED = 32     /* given by samples: pwl_build_sampled only                                 */
} pwl_func;

typedef enum pwl_partition {
    PWL_UNIFORM = 0,   /* x_k = a + (b - a) k / N (Sec. IV, uniform case)                      */
    PWL_OPTIMAL = 1    /* quasi-optimal partition F(x_i) = i / N, density |f''|^(2/5) (Sec. III-B1) */
} pwl_partition;

typedef enum pwl_values {
    PWL_INTERP = 0,    /* linear interpolant: v_k = f(x_k) (Sec. II-B1)                 */
    PWL_PROJ = 1       /* L2 orthogonal projection: M c = b, hat basis (Sec. II-B2)     */
} pwl_values;

/* Error norms of pwl_plan_tol / pwl_build_tol. */
typedef enum pwl_norm {
    PWL_NORM_L2 = 0,    /* || f - v ||_{L2[a,b]}   */
    PWL_NORM_LINF = 1   /* max over [a, b] |f - v| */
} pwl_norm;

/* Build flags, reported by pwl_table_check and pwl_table_info. */
#define PWL_FLAG_DEGENERATE 1       /* f'' == 0 everywhere: optimal partition fell back to uniform */
#define PWL_FLAG_KNOTS_COLLAPSED 2  /* FP32 knots not strictly increasing: table unusable (NaN)    */
#define PWL_FLAG_NONFINITE 4        /* the density integral was not finite: uniform fallback       */

typedef struct pwl_table pwl_table;
typedef struct pwl_batch pwl_batch;

/* ---- tables ----------------------------------------------------------- */

/*
 * pwl_build - allocate a table and enqueue its construction on `stream`.
 *   func, params[nparams]  the function f (see pwl_func); nparams in [0, 6].
 *   a < b                  the domain; both are rounded to FP32 first and the
 *                          rounded values are the table's domain.
 *   N                      number of segments, 1 <= N <= PWL_MAX_N.
 *   partition              PWL_UNIFORM, or PWL_OPTIMAL: the knots x_i solve
 *                          F(x_i) = i/N where F is the normalised cumulative
 *                          integral of |f''|^(2/5) (Sec. III-B1, the
 *                          equations for the local knot density, the
 *                          partition and F).  F is discretised on M = 256 N
 *                          cells with the trapezoid rule and an FP64 prefix
 *                          scan, inverted linearly inside the cell that
 *                          reaches i S_M / N; knots are rounded to FP32.
 *   values                 PWL_INTERP: v_k = f(x_k); PWL_PROJ: c solves
 *                          M c = b with m_ij = <phi_i, phi_j>, b_i = <f, phi_i>
 *                          (Sec. II-B2); b by 16-point Gauss-Legendre per
 *                          segment, the tridiagonal solve in FP64.
 *   out                    receives the table (library-owned).
 * Returns PWL_EINVAL for bad arguments, PWL_ECAPACITY for N > PWL_MAX_N,
 * PWL_ENOMEM / PWL_EHIP on device failures.  Knot collapse is only known
 * once the build has run: see pwl_table_check.
 */
pwl_status pwl_build(int32_t func, const double* params, int32_t nparams, double a, double b,
                     int32_t N, int32_t partition, int32_t values, void* stream, pwl_table** out);

/*
 * pwl_build_sampled - a table for any f given by samples: f_i = f(t_i) and
 * f2_i = f''(t_i) at t_i = a + i (b - a) / S, i = 0..S (DEVICE FP64 arrays of
 * S + 1 values, S >= 1).  Between samples f is the cubic spline with those
 * values and second derivatives (on [t_i, t_{i+1}], u = (x - t_i) / h:
 * (1-u) f_i + u f_{i+1} - h^2 u (1-u) ((2-u) f2_i + (1+u) f2_{i+1}) / 6), so
 * f'' is the linear interpolant of f2 - the density of the optimal
 * partition (Sec. III-B1) and the values follow as for the built-in
 * functions.  The other arguments are as in pwl_build (the table domain is
 * [a, b] rounded to FP32).  The build enqueued on `stream` reads the
 * samples: keep them alive until it has run (pwl_table_check synchronises).
 * A sampled table cannot be rebuilt with pwl_rebuild (PWL_EINVAL): build a
 * new one.
 */
pwl_status pwl_build_sampled(const double* f, const double* f2, int32_t S, double a, double b, int32_t N,
                             int32_t partition, int32_t values, void* stream, pwl_table** out);

/*
 * pwl_plan_tol - the number of segments N and the partition that reach a
 * target error `tol` in `norm` for the given values kind, from the error
 * predictions the paper derives for smooth f (Sec. III-B2): with
 * I = int |f''|^(2/5) over [a, b],
 *   L2, interpolant:  optimal I^(5/2) / (N^2 sqrt(120))             (Result 4)
 *                     uniform (b-a)^2 ||f''||_2 / (N^2 sqrt(120))    (Result 6)
 *   L2, projection:   the same divided by sqrt(6)                     (Result 5)
 *   L-infinity (not in the paper; from the interpolation remainder and the
 *   projection's element minimisers): optimal max|f''|^(1/5) I^2 / (k N^2),
 *   uniform (b-a)^2 max|f''| / (k N^2), k = 8 (interpolant), 12 (projection).
 * The integrals are computed on the GPU (FP64, trapezoid rule on 2^20
 * cells).  N is the smallest integer whose prediction is <= tol for either
 * partition; the optimal partition is chosen only when it needs fewer
 * segments.  These are asymptotic estimates (within a few percent once the
 * segments resolve f''; N >= 256 for the functions here; the projection's
 * L-infinity error runs up to ~10% above its estimate), and they describe
 * the exact CPWL: the FP32 table adds ~1e-7 max|f| (the projection's FP32
 * quadrature up to ~2e-7), so targets near 1e-6 max|f| and below are met
 * only up to that floor.  Outputs are
 * nullable: N, the partition, the predicted error at that N.  Synchronises
 * `stream`; allocates and frees a small device buffer.  Returns
 * PWL_ECAPACITY (message: the N needed) when N would exceed PWL_MAX_N, and
 * N = 1 with a predicted error of 0 when f'' vanishes (affine f).
 */
pwl_status pwl_plan_tol(int32_t func, const double* params, int32_t nparams, double a, double b, double tol,
                        int32_t norm, int32_t values, void* stream, int32_t* N, int32_t* partition,
                        double* predicted);

/* pwl_build_tol - pwl_plan_tol, then pwl_build with the N and partition it chose. */
pwl_status pwl_build_tol(int32_t func, const double* params, int32_t nparams, double a, double b, double tol,
                         int32_t norm, int32_t values, void* stream, pwl_table** out);

/*
 * pwl_rebuild - enqueue a new construction into an existing table, reusing
 * its device memory.  The table keeps its N; every other argument is as in
 * pwl_build.  The caller must not evaluate the table on another stream
 * while the rebuild is in flight.
 */
pwl_status pwl_rebuild(pwl_table* t, int32_t func, const double* params, int32_t nparams, double a,
                       double b, int32_t partition, int32_t values, void* stream);

/*
 * pwl_table_check - synchronise `stream` and report the table's build flags
 * (PWL_FLAG_*) in *flags (nullable).  Returns PWL_EKNOTS if the FP32 knots
 * collapsed (the table then evaluates to NaN), PWL_OK otherwise.
 */
pwl_status pwl_table_check(const pwl_table* t, void* stream, int32_t* flags);

/*
 * pwl_table_info - description of a table.  Every output pointer is
 * nullable.  map_cells is the number of cells of the uniform index map the
 * evaluator uses to locate segments: 2N for a uniform partition; 4N for the
 * optimal one, or 8N (N <= 2048) when the host predicts from f'' that 4N
 * cells would hold three knots where they crowd.  It affects speed only: the
 * map locates exactly for any size.  flags receives the PWL_FLAG_* word of
 * the table's last build (PWL_FLAG_DEGENERATE when f'' vanished and the
 * optimal partition fell back to uniform, PWL_FLAG_KNOTS_COLLAPSED, ...):
 * asking for it waits for that build to finish - on a library-internal
 * stream, for an event recorded after the build, not for the caller's
 * streams - and reads one word from the device.  Every other output is
 * host-side and needs no device access.
 */
pwl_status pwl_table_info(const pwl_table* t, int32_t* N, double* a, double* b, int32_t* partition,
                          int32_t* values, int32_t* map_cells, int32_t* flags);

/*
 * pwl_table_download - copy the table to HOST buffers (each nullable):
 * knots[N+1] FP32 knots, values[N+1] FP32 vertex values, knots64[N+1] FP64
 * knots before rounding, values64[N+1] FP64 vertex values (for PWL_PROJ the
 * FP64 solution of M c = b; for PWL_INTERP the FP32 values widened).
 * Synchronises `stream`.
 */
pwl_status pwl_table_download(const pwl_table* t, float* knots, float* values, double* knots64,
                              double* values64, void* stream);

/* pwl_table_free - release a table (waits for the device to finish with it). NULL is a no-op. */
void pwl_table_free(pwl_table* t);

/* ---- evaluation (Algorithm 1, Sec. IV) --------------------------------- */

/*
 * pwl_eval - y[i] = v(x[i]) for i < n.
 *   v_override  nullable device [N+1] FP32 vertex values used instead of the
 *               table's own (slopes are then derived from them on the fly).
 *   x, y        device FP32 [n]; y may not alias x partially (y == x is allowed).
 */
pwl_status pwl_eval(const pwl_table* t, const float* v_override, const float* x, float* y, int64_t n,
                    void* stream);

/*
 * pwl_eval_backward - fused forward and backward of pwl_eval for an upstream
 * gradient g: y = v(x) (nullable), dx = g * v'(x) (nullable; 0 where x was
 * clamped, the left slope at x = b), dv[k] = sum over points of g times the
 * hat weight phi_k(x) (nullable; device [N+1]; OVERWRITTEN: each workgroup
 * sums its points in FP64 and writes the sums, rounded to FP32, as one row
 * of a per-table workspace; a second kernel adds the rows in FP64 in a fixed
 * order, so dv is deterministic for a given launch shape).  At least one of
 * y, dx, dv must be non-NULL.  This is the exact derivative of Algorithm 1
 * (the paper gives none): dy/dx is the segment slope, dy/dv_k the hat weight.
 * Workspace: (workgroups x (N+1)) floats owned by the table, taken from
 * the stream-ordered allocator (hipMallocAsync on `stream`) by the first
 * call with dv that needs more; the old rows are released on `stream` after
 * their last user has finished, and the rows are freed with the table.
 * Calls with dv on one table share them, so they must not overlap in time:
 * issue them on one stream.
 */
pwl_status pwl_eval_backward(const pwl_table* t, const float* v_override, const float* x,
                             const float* g, float* y, float* dx, float* dv, int64_t n, void* stream);

/*
 * pwl_eval_backward_noalloc - pwl_eval_backward for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same kernels, launch shape
 * and results (bit-identical outputs), but the dL/dv partial sums live in a
 * fixed device array of the library (8 MiB, 2^21 floats per device, held
 * until the process ends) instead of a workspace of the table.  It calls no
 * allocation routine.  Arguments are as in pwl_eval_backward.  Returns
 * PWL_ECAPACITY, enqueuing nothing, when dv is requested and the launch
 * needs more than 2^21 floats (workgroups x (N + 1); the default backward
 * shape needs at most 256 x 4097 on a 256-CU device).  Every call on a
 * device shares that device's array: calls with dv that overlap in time on
 * one device (other streams, other threads) race and give wrong gradients,
 * so issue them on one stream.  The table must have been built (that first
 * library call on the device does the one-time set-up).
 */
pwl_status pwl_eval_backward_noalloc(const pwl_table* t, const float* v_override, const float* x,
                                     const float* g, float* y, float* dx, float* dv, int64_t n,
                                     void* stream);

/*
 * pwl_locate - the 0-based segment index i with x_i <= x < x_{i+1} of each
 * point (the segment locate of Algorithm 1), after clamping to [a, b]; x = b gives N-1,
 * NaN gives 0.  seg is device int32 [n].  It runs the very locate the
 * evaluation kernels run for this table (the same unrolled compare depth, or
 * the binary search when pwl_set_locate selected it), so the indices are
 * those pwl_eval, pwl_eval_backward and the batched kernels use.
 */
pwl_status pwl_locate(const pwl_table* t, const float* x, int32_t* seg, int64_t n, void* stream);

/* ---- batches of tables ------------------------------------------------- */

/*
 * pwl_batch_create - prepare the launches that evaluate T tables, table t on
 * the points [offsets[t], offsets[t+1]) of concatenated point arrays.
 *   tables[T]    tables on the current device.  The batch copies each
 *                table's evaluation data (records, knots, index map) into
 *                its own memory here, so the tables may be freed or rebuilt
 *                afterwards without affecting it (a rebuilt table needs a
 *                new batch to be seen).
 *   offsets[T+1] HOST array, offsets[0] = 0, non-decreasing (empty tables
 *                allowed); offsets[T] is the total number of points.
 * Each direction is one launch, planned for the PWL_KERNEL_BATCH (forward)
 * or PWL_KERNEL_BATCH_BACKWARD launch shape current at creation.
 * Forward: the points are cut into slices of two of the kernel's vector
 * iterations (unroll * block * 8 points) from point 0 on, whatever the
 * tables; a slice whose tables' LDS images do not fit together is split at
 * a table.  The grid holds wg_per_cu workgroups per CU (fewer if there are
 * fewer slices) and workgroup b takes the slices at launch positions b,
 * b + grid, ... (runs of 8 consecutive slices are placed on one XCD): per
 * slice it copies the images of the slice's tables into LDS and streams the
 * slice as one range, each wave with the table of its points.
 * Backward: the same, in slices of four of its own iterations
 * (unroll * block * 16 points); per slice the
 * workgroup also sums every point's hat weights into one FP64 dL/dv region
 * per table in LDS and stores each region, rounded to FP32, as that run's
 * N + 1 partial sums in a buffer the batch owns; a second kernel adds each
 * table's partial sums in slice order in FP64.
 * Packs the copies, uploads the plan and synchronises `stream`.
 */
pwl_status pwl_batch_create(const pwl_table* const* tables, int32_t T, const int64_t* offsets, void* stream,
                            pwl_batch** out);

/* pwl_batch_eval - y = v_t(x) for every table t over its points (device FP32 [offsets[T]]). */
pwl_status pwl_batch_eval(pwl_batch* bt, const float* x, float* y, void* stream);

/*
 * pwl_batch_eval_backward - fused forward + backward for every table: y and
 * dx (each nullable) as in pwl_eval_backward; g is required unless the
 * batch has no points; dv (required) is the concatenation of every table's
 * N_t + 1 gradients, table t first, and is OVERWRITTEN (zero for tables
 * without points).  The slices' partial sums are added in a fixed order,
 * so dv does not depend on the order in which workgroups ran (within a
 * slice the FP64 LDS sums depend on it only in their last FP64 bits).  The
 * partial sums live in the batch: calls on one batch must not overlap (on
 * different streams, or with a replay of its graph).
 */
pwl_status pwl_batch_eval_backward(pwl_batch* bt, const float* x, const float* g, float* y, float* dx,
                                   float* dv, void* stream);

/*
 * pwl_batch_capture - record the launch sequence of pwl_batch_eval (g NULL)
 * or pwl_batch_eval_backward (g non-NULL) for these exact buffers into a HIP
 * graph owned by the batch (replacing a previous one); pwl_batch_replay
 * launches it on `stream`.  The graph uses no memset nodes (dv is cleared by
 * a kernel).  Capture synchronises `stream`.
 */
pwl_status pwl_batch_capture(pwl_batch* bt, const float* x, const float* g, float* y, float* dx, float* dv,
                             void* stream);
pwl_status pwl_batch_replay(pwl_batch* bt, void* stream);

/*
 * pwl_batch_info - shape of a batch (outputs nullable): tables, points, dv
 * length, and per direction the workgroups and table runs of its launch
 * (the forward's runs: one per table per slice it meets).
 */
pwl_status pwl_batch_info(const pwl_batch* bt, int32_t* T, int64_t* npoints, int64_t* dv_len, int32_t* grid_fwd,
                          int32_t* grid_bwd, int32_t* runs_fwd, int32_t* runs_bwd);

/* pwl_batch_free - release a batch and its graph. NULL is a no-op. */
void pwl_batch_free(pwl_batch* bt);

/* ---- baselines and probes ----------------------------------------------- */

/*
 * pwl_direct_gaussian - y = amp * exp(-x^2 / (2 s^2)) computed directly with
 * the device math library (fast != 0 selects the reduced-precision
 * exponential), the comparison the paper makes in Sec. VI-A.
 */
pwl_status pwl_direct_gaussian(const float* x, float* y, int64_t n, float s, float amp, int32_t fast,
                               void* stream);

/*
 * pwl_direct_eval - y = f(x) evaluated directly in FP32 with the device math
 * library (expf, j0f, IEEE division; no table): the baseline each table is
 * compared with (Sec. VI).  func and params as in pwl_build (not
 * PWL_F_SAMPLED); x, y device FP32 [n].
 */
pwl_status pwl_direct_eval(int32_t func, const double* params, int32_t nparams, const float* x, float* y, int64_t n,
                           void* stream);

/* pwl_copy - dst = src (device FP32 [n]); the HBM bandwidth probe. */
pwl_status pwl_copy(const float* src, float* dst, int64_t n, void* stream);

/* ---- sample application ------------------------------------------------- */

#define PWL_KDE_TABLE 0       /* kernel values through the table                 */
#define PWL_KDE_EXPF 1        /* expf                                             */
#define PWL_KDE_FAST_EXPF 2   /* __expf                                           */

/*
 * pwl_kde - per-pixel sums of Gaussian kernels of a nonparametric background
 * model, the application the paper accelerates with its tables (Sec. VI-A):
 *   out[y, x] = 1 / (T (2r+1)^2) * sum over k < T and the (2r+1)^2 window of
 *               (y, x) (clamped to the image) of
 *               prod_{c = 0, 1, 2} g((frame[y, x, c] - hist[k, y', x', c]) / sigma[c]),
 * g(u) = exp(-u^2 / 2).  frame is DEVICE RGBA8 [H, W, 4], hist DEVICE RGBA8
 * [T, H, W, 4] (alpha ignored), sigma a HOST array of 3 positive values, out
 * DEVICE FP32 [H, W].  mode PWL_KDE_TABLE evaluates g through `t` (a table
 * of exp(-u^2/2); its argument is |u| when the table's domain starts at 0,
 * so a table on [0, 8] serves, as in the paper); the other modes ignore `t`
 * (may be NULL).  1 <= H, W; 1 <= T; 0 <= r <= 32.  Sums are accumulated in
 * FP64; each kernel value is FP32.
 */
pwl_status pwl_kde(const pwl_table* t, int32_t mode, const void* frame, const void* hist, int32_t H, int32_t W,
                   int32_t T, int32_t r, const float* sigma, float* out, void* stream);



/* ---- launch tuning -------------------------------------------------------- */

#define PWL_KERNEL_FORWARD 0    /* pwl_eval, pwl_locate   */
#define PWL_KERNEL_BACKWARD 1   /* pwl_eval_backward      */
#define PWL_KERNEL_BATCH 2      /* the batched forward    */
#define PWL_KERNEL_BATCH_BACKWARD 3   /* the batched fused backward */

/*
 * pwl_set_launch - process-wide launch shape of one evaluation kernel family:
 * each thread streams `unroll` (1, 2 or 4) 16-byte vectors per iteration,
 * workgroups have `block` threads (a multiple of 64 in [64, 1024]) and the
 * grid holds up to `wg_per_cu` (1..32) of them per compute unit, more than
 * can be resident at once if asked (later ones start as earlier ones end).
 * The batched forward's grid is persistent: its workgroups take the
 * batch's slices round-robin.
 * The single-table kernels cut the grid back, a whole workgroup per compute
 * unit at a time and to no fewer than one per compute unit, until each
 * workgroup streams at least 2^15 points and 2 points per byte of the table
 * it stages in LDS.  All three
 * zero restores the default.  Used by the autotuner; takes effect for later
 * launches.
 * pwl_get_launch reads the current shape back (outputs nullable).
 */
pwl_status pwl_set_launch(int32_t kernel, int32_t unroll, int32_t block, int32_t wg_per_cu);
pwl_status pwl_get_launch(int32_t kernel, int32_t* unroll, int32_t* block, int32_t* wg_per_cu);

#define PWL_LOCATE_MAP 0      /* uniform index map + unrolled compares (default)              */
#define PWL_LOCATE_SEARCH 1   /* branch-free binary search over the knots in LDS (Sec. IV-V)  */

/*
 * pwl_set_locate - process-wide segment locate of pwl_eval (the first
 * part of Algorithm 1): the index map, or the paper's own GPU technique, a binary
 * search unrolled into selects, over the knots staged in LDS (no map).
 * Both give the same segment, so the outputs are bit-identical; the choice
 * is a speed A/B.  Takes effect for later launches.  pwl_get_locate reads
 * the mode back.
 */
pwl_status pwl_set_locate(int32_t mode);
int32_t pwl_get_locate(void);

#define PWL_RECORDS_PACKED 0  /* one 16-byte record {x_k, v_k, slope_k, x_{k+1}} per segment (default) */
#define PWL_RECORDS_SOA 1     /* the same fields as four arrays of N floats                        */
#define PWL_RECORDS_PAIRS 2   /* 8-byte {v_k, slope_k} pairs; x_k from the knot array              */

/*
 * pwl_set_records - process-wide arrangement of the per-segment data that
 * pwl_eval stages in LDS (Sec. V discusses arranging the table for the
 * GPU's memory): packed records, where a point's lookup is one 12-byte LDS
 * read; structure-of-arrays, three 4-byte reads; or value/slope pairs, one
 * 8-byte read, the segment's knot coming from the knot reads of the locate
 * (the smallest image: 8 bytes per segment instead of 16).  The values are
 * the same, so outputs are bit-identical; the choice is a speed A/B.  The
 * fused backward, the batched kernels and pwl_kde always use packed
 * records.  Takes effect for later launches; pwl_get_records reads it back.
 */
pwl_status pwl_set_records(int32_t layout);
int32_t pwl_get_records(void);

/* ---- library ------------------------------------------------------------ */

const char* pwl_last_error(void);
int32_t pwl_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PWL_H */
