/*
 * h2s.h -- C ABI of the MI355X H2* / (H2+H)* fast kernel matrix-vector product.
 *
 * Method: Khan & Ambikasaran, "New algebraic fast algorithms for N-body
 * problems in two and three dimensions" (arXiv 2309.14085).
 *   build  -- uniform 2^d tree (Sec. 3.1), weak-admissibility lists (Sec. 3.3,
 *             Table "HOD_notation"), B2T NCA on the far field and T2B NCA on
 *             the vertex-sharing field (Sec. 5.1.1, Algs. "b2t" / "t2b"), or
 *             per-pair ACA on the vertex-sharing field for (H2+H)* (Sec. 5.2.1,
 *             Alg. "pure_aca"), and the operators of Sec. 3.4.3.  Runs on the
 *             host in C++; the operators are then copied to device memory.
 *   apply  -- phi = K~ x (Sec. 5.1.2, Sec. 5.2.2): P2M, M2M, M2L, L2L, L2P and
 *             the direct near field, all in HIP kernels on the caller's stream.
 *
 * Conventions
 *   - Every call returns h2s_status; no C++ exception crosses the ABI.
 *   - Arguments are validated before anything is allocated.  On failure an
 *     output handle is set to NULL, nothing leaks, and h2s_last_error() gives a
 *     thread-local description.
 *   - Points are host memory, row-major n x d doubles.  x and y of apply are
 *     DEVICE pointers, user (input) order, column-major n x nrhs doubles with
 *     leading dimensions ldx, ldy >= n.  The library never frees or retains
 *     caller memory.
 *   - `stream` is a hipStream_t (NULL = the null stream).  apply is
 *     asynchronous with respect to the host and ordered on `stream`; a kernel
 *     fault surfaces at the caller's next synchronisation of that stream.
 *   - One handle may be used by one stream at a time (its device workspace is
 *     shared by its calls); distinct handles may run concurrently.
 */
#ifndef H2S_H
#define H2S_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    H2S_OK = 0,
    H2S_ERR_INVALID_ARG = 1,
    H2S_ERR_OUT_OF_MEMORY = 2,
    H2S_ERR_DEVICE = 3,
    H2S_ERR_NOT_CONVERGED = 4,
    H2S_ERR_UNSUPPORTED = 5,
    H2S_ERR_INTERNAL = 6
} h2s_status;

/* Kernel functions of r = |x-y|.  LOG_R: log r (2D single-layer Laplacian,
 * Sec. 6.1.1); INV_R: 1/r (3D single-layer Laplacian, Sec. 6.2.1); GAUSSIAN:
 * exp(-r^2 / param^2) (RBF interpolation); EXP_R: exp(-r) (Matern nu = 1/2,
 * Appendix D); RBF_AR: a/r for r >= a, r/a for r < a (2D RBF interpolation,
 * Sec. 6); RBF_LOG: log r / log a for r >= a, (r log r - 1)/(a log a - 1) for
 * r < a (3D RBF interpolation, Sec. 6); a = param.  NTI_MQ: the non-
 * translation-invariant scaled multiquadric (r^2 + (c(x) - c(y))^2 + 1)^(3/2)
 * with c(x) = exp(-(x_1 + x_3)) (3D RBF interpolation, Sec. 6); d = 3 only,
 * not with H2S_FP32_M2L.  The closed set is compiled into the device code. */
typedef enum {
    H2S_K_LOG_R = 0,
    H2S_K_INV_R = 1,
    H2S_K_GAUSSIAN = 2,
    H2S_K_EXP_R = 3,
    H2S_K_RBF_AR = 4,
    H2S_K_RBF_LOG = 5,
    H2S_K_NTI_MQ = 6
} h2s_kernel_kind;

typedef struct {
    h2s_kernel_kind kind;
    double param; /* GAUSSIAN length scale h > 0; radius a > 0 of RBF_AR / RBF_LOG (a != 1 for RBF_LOG) */
    double diag;  /* K(x, x), used whenever two points coincide: 0 for LOG_R / INV_R (Sec. 6.1.1, 6.2.1) and the RBFs */
    double shift; /* the matrix is K + shift * I */
} h2s_kernel;

typedef enum { H2S_H2STAR = 0, H2S_H2_PLUS_H = 1 } h2s_variant;

/* Internal arithmetic of apply; x and y stay double at the boundary.
 *   FP64      everything in double.
 *   FP32      near field (kernel evaluations with box-centred coordinates)
 *             and leaf bases in float; M2L, transfers, multipole and local
 *             coefficients and every accumulation in double.
 *   FP32_M2L  as FP32, and the far-field M2L evaluated in float as well (for
 *             log r as a per-pair constant in double plus a float remainder).
 *             The interpolative operators amplify float M2L values, so its
 *             error against FP64 is larger; it is reported, not bounded.  In
 *             products of several right-hand sides (blocks of 8 columns) the
 *             far-field M2L runs on the matrix cores in float
 *             (v_mfma_f32_16x16x4f32), kernel values shared by 32 columns.
 *   FP32_BF16M2L  as FP32_M2L, and in products of several right-hand sides
 *             the far-field kernel values and multipoles enter the matrix
 *             cores as bfloat16 (v_mfma_f32_16x16x32_bf16, float accumulation).
 *             Single-column products are FP32_M2L's.  Its error is reported,
 *             not bounded.
 * FP32_M2L and FP32_BF16M2L are not available for the NTI multiquadric. */
typedef enum { H2S_FP64 = 0, H2S_FP32 = 1, H2S_FP32_M2L = 2, H2S_FP32_BF16M2L = 3 } h2s_precision;

typedef struct {
    int32_t leaf_size;    /* n_max >= 1: leaf level kappa = ceil(log_{2^d}(n / n_max)) (Sec. 3.1) */
    double eps_far;       /* ACA tolerance of the far-field NCA, >= 0 (Sec. 5.1.1) */
    double eps_ver;       /* ACA tolerance of the vertex-sharing NCA / per-pair ACA, >= 0 */
    h2s_variant variant;
    h2s_precision prec;
    int32_t host_threads; /* OpenMP threads for the host build; <= 0 = runtime default */
    int32_t host_only;    /* 1: build the representation on the host only (export / stats; apply is rejected) */
    int64_t hbm_budget_bytes; /* the most device memory the handle may ever hold (representation, product
                                 and solve buffers, allocated on first use); an allocation beyond it fails
                                 as OUT_OF_MEMORY like a failed hipMalloc.  <= 0: no limit */
} h2s_build_opts;

typedef struct h2s_tree_s *h2s_tree;

/* Build the representation of the n x n kernel matrix of `points`.
 * points: host, row-major n x d doubles (copied).  d in {2, 3}; n >= 1; all
 * coordinates finite.  The handle owns all device memory until h2s_free.
 * Errors: INVALID_ARG (bad argument), OUT_OF_MEMORY (host or device, or
 * opts->hbm_budget_bytes too small for the representation; nothing leaks),
 * DEVICE (no HIP device / HIP error), UNSUPPORTED (a leaf of more than 4096
 * points, a stacked transfer of more than 2560 rows, a rank above 512 or an
 * interaction list of more than 256 boxes: the kernels stage these whole in
 * LDS), INTERNAL. */
h2s_status h2s_build(const double *points, int64_t n, int32_t d, const h2s_kernel *kernel,
                     const h2s_build_opts *opts, void *stream, h2s_tree *out);

/* y = (K~ + shift I) x for nrhs right-hand sides (Sec. 5.1.2 / 5.2.2).
 * x, y: device, user order, column-major, ld >= n; x and y must not overlap.
 * Asynchronous and ordered on `stream`: the direct near field runs on a
 * second stream owned by the handle, forked from and joined back into
 * `stream` with events, so the caller sees one stream-ordered operation.
 * One handle serves one stream at a time.
 * Errors: INVALID_ARG, UNSUPPORTED (host_only handle), DEVICE. */
h2s_status h2s_apply(h2s_tree t, const double *x, double *y, int32_t nrhs, int64_t ldx, int64_t ldy,
                     void *stream);

/* Phase masks for h2s_apply_phases. */
#define H2S_PHASE_NEAR 1u /* direct near field N* plus shift * x (Sec. 5.1.2, near-field potential) */
#define H2S_PHASE_FAR 2u  /* far field through the nested far basis */
#define H2S_PHASE_VER 4u  /* vertex-sharing field: nested basis (H2*) or per-pair low rank ((H2+H)*) */
#define H2S_PHASE_ALL 7u

/* As h2s_apply, restricted to the phases in `mask` (non-zero subset of
 * H2S_PHASE_ALL); used to check each part of the product separately. */
h2s_status h2s_apply_phases(h2s_tree t, uint32_t mask, const double *x, double *y, int32_t nrhs,
                            int64_t ldx, int64_t ldy, void *stream);

/* Options of h2s_solve.  h2s_solve_opts_default fills the defaults shown. */
typedef struct {
    int32_t restart;          /* GMRES restart length m, 1..1000 (50) */
    int32_t max_iter;         /* Krylov steps over all cycles (10000) */
    int32_t max_refine;       /* refinement steps = GMRES cycles (1000) */
    h2s_precision inner_prec; /* precision of the products inside the Krylov cycles (H2S_FP32) */
    double rtol;              /* target ||b - K~ x|| / ||b|| with the FP64 product (1e-8) */
    double inner_rtol;        /* a cycle stops once its residual estimate falls by this factor (1e-6) */
    int32_t use_x0;           /* 1: x holds the initial guess on entry; 0: start from x = 0 (0) */
} h2s_solve_opts;

typedef struct {
    int32_t iterations;  /* Krylov steps (products in the inner precision) */
    int32_t refinements; /* refinement steps (FP64 residual products) */
    int32_t converged;   /* 1 if the FP64 relative residual reached rtol */
    double residual;     /* final ||b - K~ x|| / ||b|| with the FP64 product */
} h2s_solve_info;

h2s_status h2s_solve_opts_default(h2s_solve_opts *opts);

/* Solve (K~ + shift I) x = b for nrhs right-hand sides, one after another:
 * GMRES with iterative refinement (Sec. 6: GMRES on the fast product to a
 * relative residual tolerance).  Each refinement step computes the FP64
 * residual r = b - K~ x and runs one GMRES(restart) cycle on K~ d = r with the
 * products in opts->inner_prec; Arnoldi vectors, both classical Gram-Schmidt
 * passes, norms and the update x += d stay in FP64 on the device.
 * b, x: device, user order, column-major, ld >= n; must not overlap.
 * opts: NULL for the defaults.  info: NULL or nrhs entries.
 * The handle uploads the FP64 and the inner-precision representations on
 * first use (whatever its build precision) and keeps an n x (restart + 1)
 * FP64 workspace.  Returns H2S_ERR_NOT_CONVERGED, with x the last iterate
 * and info filled, when some right-hand side misses rtol within max_iter or
 * max_refine steps or stagnates (three cycles without a 0.1% gain).
 * Synchronises `stream` once per Krylov step.
 * Errors: INVALID_ARG, UNSUPPORTED (host_only handle), OUT_OF_MEMORY, DEVICE,
 * NOT_CONVERGED. */
h2s_status h2s_solve(h2s_tree t, const double *b, double *x, int32_t nrhs, int64_t ldb, int64_t ldx,
                     const h2s_solve_opts *opts, h2s_solve_info *info, void *stream);

/* Release the handle and its device memory (NULL is accepted). */
h2s_status h2s_free(h2s_tree t);

typedef struct {
    int32_t d, kappa, variant, prec;
    int64_t n;
    int64_t boxes;                /* non-empty boxes over all levels */
    int64_t near_pairs;           /* ordered leaf pairs in the near lists (self included) */
    int64_t far_pairs, ver_pairs; /* ordered box pairs over all levels */
    int64_t rank_sum[2];          /* sum of ranks, far / vertex family */
    int32_t rank_max[2];
    int64_t p2p_evals;            /* kernel evaluations of the near field */
    int64_t m2l_evals;            /* kernel evaluations of M2L (sum of r_X r_Y) */
    int64_t m2l_evals_family[2];  /* the same for the far / vertex family */
    int64_t leaf_basis_entries;   /* sum over leaves and families of n_X r_X (P2M / L2P operators) */
    int64_t transfer_entries;     /* sum over non-leaf boxes and families of (sum_c r_c) r_X */
    int64_t pair_entries;         /* (H2+H)*: sum over vertex pairs of (n_X + n_Y) r */
    int64_t operator_bytes;       /* stored operators on the device */
    int64_t device_bytes;         /* all device memory the handle owns */
    double build_seconds;         /* host build wall time */
    int32_t rank_max_level[2][32];
    double rank_avg_level[2][32];
    int64_t leaf_basis_stored;    /* leaf-basis entries stored on the device (rows other than exact unit rows), one copy */
    int64_t transfer_stored;      /* the same for the stacked transfers */
} h2s_stats;

/* Sizes, ranks per level and work counts of a handle. */
h2s_status h2s_get_stats(h2s_tree t, h2s_stats *s);

/* Write the tree, permutation, lists, pivots and FP64 operators to `path` as a
 * container of named arrays: the bytes "H2SX", uint32 version (1), uint32
 * array count, then per array a NUL-padded char name[32], uint32 dtype
 * (1 = int32, 2 = int64, 3 = float64), uint32 ndim, int64 dims[ndim] and the
 * little-endian data.  Arrays: meta (d, kappa, n, variant), cube (centre,
 * half-width), perm, points (tree order), lev_off, box_begin / end / parent /
 * coord / morton, {near,far,ver}_off / _idx, and per family fam_{far,ver}_
 * rank / coef_off / piv_row / piv_col / op_off / op_rows / op (leaf U_X
 * column-major, stacked L2L row-major), pairs (level, x, y, rank, off_u,
 * off_v per (H2+H)* pair) and pair_data. */
h2s_status h2s_export(h2s_tree t, const char *path);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc.  The same
 * product as h2s_apply through the batched multi-RHS kernels (blocks of 8
 * columns), for 1 <= nrhs <= 32, with the batch buffers (charges, near-field
 * potentials, multipoles and locals of the active blocks) in a file-scope
 * device array of H2S_NOALLOC_SCRATCH_BYTES per GPU instead of buffers the
 * handle allocates on its first multi-RHS product.  The results equal
 * h2s_apply's for the same nrhs > 1 bit for bit.  The array is shared by
 * every call on one GPU and keeps the last call's contents (every call writes
 * all it reads), so calls that overlap on one GPU race: order them on one
 * stream.  The handle's auxiliary streams are created on its first product
 * of any kind (streams and events, no device memory).
 * Requirements: an H2* handle of precision FP64 or FP32; ceil(nrhs / 8) * 64 *
 * (2 n + 2 (far + vertex coefficients)) bytes <= H2S_NOALLOC_SCRATCH_BYTES.
 * Errors: INVALID_ARG (as h2s_apply, or nrhs > 32), UNSUPPORTED (variant,
 * precision, host_only handle, or a size beyond the array), DEVICE. */
#define H2S_NOALLOC_SCRATCH_BYTES (256u << 20)
h2s_status h2s_apply_noalloc(h2s_tree t, const double *x, double *y, int32_t nrhs, int64_t ldx, int64_t ldy,
                             void *stream);

/* Measurement: the peak rate R_eval of the device kernel function, the
 * ceiling of the phases that evaluate kernel values on the fly (the near
 * field of Sec. 5.1.2 and the M2L blocks T_{X,Y} = K(t^{X,i}, t^{Y,i}) of
 * Sec. 3.4.3).  A register-resident loop: every thread holds 4 targets and 8
 * sources in registers and sums K(x, y) q over them pass after pass, with the
 * lookup table of the table-driven functions in LDS as in the product
 * kernels, so nothing but the evaluation itself limits it.  kernel: kind and
 * param as for h2s_build (diag and shift unused); d in {2, 3} (3 for the NTI
 * multiquadric); prec H2S_FP64 (the double functions of the FP64 product) or
 * H2S_FP32 (the float functions of the FP32 near field).  Writes the fastest
 * of five timed launches, in evaluations per second, to *evals_per_s.
 * Synchronises `stream`; allocates and frees a small device buffer.
 * Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE. */
h2s_status h2s_eval_rate(const h2s_kernel *kernel, int32_t d, int32_t prec, double *evals_per_s, void *stream);

/* Kernel classes timed by the profiling hooks, in launch order. */
#define H2S_PROF_LEAF_UP 0   /* charges to tree order + P2M */
#define H2S_PROF_M2M 1       /* all M2M levels */
#define H2S_PROF_M2L_FAR 2   /* far-field M2L, every level in one launch */
#define H2S_PROF_L2L 3       /* all L2L levels */
#define H2S_PROF_PAIR_PART 4 /* (H2+H)* partial products */
#define H2S_PROF_PAIR_SUM 5  /* (H2+H)* chunk sums */
#define H2S_PROF_LEAF_DOWN 6 /* L2P + (H2+H)* vertex blocks + sum + scatter */
#define H2S_PROF_M2L_VER 7   /* vertex-sharing M2L, every level in one launch */
#define H2S_PROF_NEAR 8      /* direct near field (beside the sweeps on a second stream when not profiling) */
#define H2S_NUM_PROF 9

/* Profiling hooks for measurement: while enabled, every apply runs all its
 * kernels on the caller's stream (the near field does not overlap the tree
 * sweeps) and records a HIP event before and after each kernel class, so
 * each class is timed alone (adding small gaps between kernels).  h2s_get_profile waits for the recorded
 * events, writes per-class total milliseconds and launch counts (arrays of
 * H2S_NUM_PROF entries, either may be NULL) and clears the record. */
h2s_status h2s_set_profiling(h2s_tree t, int32_t enable);
h2s_status h2s_get_profile(h2s_tree t, double *ms_total, int64_t *launches);

/* Launch schedule of the single-column product.  No field changes a result:
 * every P2M / M2M / L2L output is summed by one thread in index order
 * whatever the block width, and a leaf's near field is the same whichever
 * launch and stream take it, so products are equal bit for bit under any
 * valid schedule.  Entries of up_threads / dn_threads beyond level kappa
 * (h2s_stats.kappa) are ignored. */
typedef struct {
    double near_first;       /* share of the leaves (0..1) whose near field runs on the second stream
                                beside P2M and M2M; the rest runs beside L2L.  Default 0.8 */
    int32_t up_threads[33];  /* block width of P2M (level kappa) and M2M (levels 1..kappa-1):
                                a multiple of 64 in [64, 512]; default: outputs of the widest box */
    int32_t dn_threads[33];  /* block width of L2L (levels 1..kappa-1), same rule */
    int32_t m2l_stream;      /* 1: the leaf-level M2L runs on a third stream from the end of P2M, beside
                                the coarse M2M levels; 2: as 1, and the M2L of the level above the
                                leaves runs on a fourth stream as soon as M2M has made its multipoles;
                                0: all M2L after M2M.  Default 2 */
} h2s_schedule;

/* Read or replace the handle's schedule (valid on host_only handles too).
 * h2s_set_schedule rejects, with H2S_ERR_INVALID_ARG and no change, a
 * near_first outside [0, 1], an m2l_stream other than 0, 1 or 2, or a width
 * that is not a multiple of 64 in [64, 512] at any level 1..kappa.  It must not be called while another
 * call uses the handle. */
h2s_status h2s_get_schedule(h2s_tree t, h2s_schedule *s);
h2s_status h2s_set_schedule(h2s_tree t, const h2s_schedule *s);

/* Autotuner of the schedule.  Times the product y = K~ x (device vectors of
 * length n in user order, not overlapping) on stream under candidate
 * schedules: the near-field share, then the block width of every level of
 * P2M, M2M and L2L, and whether the leaf-level M2L gets its own stream, each chosen in turn with the
 * others fixed; each
 * candidate is timed twice over reps products (reps < 1 means 5) with HIP
 * events, and the faster time counts.  A candidate replaces the current
 * choice only when it is faster by more than 0.5%.  The fastest schedule is
 * installed in the handle; info (may be NULL) receives the time of the
 * schedule at entry and of the installed one (milliseconds per product) and
 * the number of candidates timed.  Synchronous: it returns after the last
 * product, and y then holds K~ x.  H2S_ERR_UNSUPPORTED for a host_only
 * handle; H2S_ERR_DEVICE if a launch or an event fails. */
typedef struct {
    double ms_entry;     /* product time with the schedule at entry */
    double ms_tuned;     /* product time with the installed schedule */
    int32_t candidates;  /* schedules timed */
} h2s_tune_info;
h2s_status h2s_tune(h2s_tree t, const double *x, double *y, int32_t reps, h2s_tune_info *info, void *stream);

/* Groups of trees applied together.  h2s_group_apply enqueues
 * y_i = K~_i x_i for every tree of the group (one right-hand side each)
 * ordered on stream.  H2* trees of one precision (H2S_FP64 or H2S_FP32),
 * kernel kind and dimension that number two or more form a fused class: one
 * kernel launch per step covers every tree of the class (permutation, near
 * field, P2M, each M2M and L2L level step, M2L per family, L2P), each block
 * taking one work item of one tree, so many trees of uneven size cost the
 * launches of one.  Every other tree's product is captured once as a HIP
 * graph (again when that tree's x[i] or y[i] pointer changes) and launched
 * on a stream of the group's own, forked from stream and joined back into it
 * with events.  A changed pointer of a fused tree makes the call wait for
 * stream before it updates the class's vector table.  The group keeps its
 * launch tables (and the block widths the trees' schedules had at creation)
 * until it is freed.  Results equal h2s_apply on each tree bit for bit.  x[i], y[i]: device vectors of tree i's n (user order), not
 * overlapping.  h2s_group_create takes count >= 1 distinct device (not
 * host_only) trees of one device; it copies the array but not the trees,
 * which must outlive the group and must not be used by another call while
 * a group apply is in flight.  Not for use under graph capture. */
typedef struct h2s_group_s *h2s_group;
h2s_status h2s_group_create(const h2s_tree *trees, int32_t count, h2s_group *out);
h2s_status h2s_group_apply(h2s_group g, const double *const *x, double *const *y, void *stream);
h2s_status h2s_group_free(h2s_group g);

/* Device memory hooks: alloc(ctx, bytes, &ptr) returns 0 on success.  NULL
 * functions restore hipMalloc / hipFree.  Affects later builds only. */
typedef int (*h2s_alloc_fn)(void *ctx, size_t bytes, void **ptr);
typedef void (*h2s_free_fn)(void *ctx, void *ptr);
h2s_status h2s_set_allocator(h2s_alloc_fn alloc_fn, h2s_free_fn free_fn, void *ctx);

const char *h2s_status_string(h2s_status s);

/* Copy the calling thread's last error text into buf (always NUL-terminated). */
h2s_status h2s_last_error(char *buf, size_t len);

#ifdef __cplusplus
}
#endif
#endif /* H2S_H */
