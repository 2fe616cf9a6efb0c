/*
 * dfacto.h -- C ABI of the MI355X (gfx950) DFacTo engine.
 *
 * The engine computes the matricized-tensor-times-Khatri-Rao product
 * (MTTKRP) of a sparse 3-way tensor the way DFacTo does (Choi &
 * Vishwanathan, "DFacTo: Distributed Factorization of Tensors", NIPS 2014,
 * Section 3, Algorithm 1): as two sparse products over a fiber-compressed
 * flattening, batched over all R rank columns, and the two solvers that sit
 * on top of it -- one CP-ALS iteration (Appendix B, Algorithm 2; Appendix E,
 * Algorithm 4) and the GD gradient (Appendix C, Algorithm 3).
 *
 * Conventions for every call:
 *  - Modes are 0-based: mode 0 = the paper's mode 1 (output rows i),
 *    mode 1 = mode 2 (rows j), mode 2 = mode 3 (rows k).
 *  - Pointers named d_* are DEVICE pointers owned by the caller; the library
 *    never frees them.  Host pointers are named h_* or are plain arrays of
 *    device pointers (d_F[3]).
 *  - Factor matrices are row-major dims[m] x R, element type given by a
 *    dfacto_dtype (FP32, or BF16 stored as raw 16-bit patterns).  Row
 *    starts must be aligned to the element size.
 *  - Work is enqueued on the stream bound to the context and is
 *    stream-ordered.  Some calls (CP-ALS, GD gradient, joint ALS) run part
 *    of their work on a second stream of the context, forked from the bound
 *    stream and joined back to it by events within the call, so the order
 *    seen from the bound stream is unchanged.  Calls that synchronize: the
 *    builds
 *    (dfacto_build_flattenings, dfacto_build_ratings), dfacto_tensor_export,
 *    the calls that return host results (dfacto_gd_step,
 *    dfacto_joint_als_iter, dfacto_profile_read, dfacto_ctx_synchronize),
 *    and a call that has to grow one of the context's workspaces (the first
 *    call at a larger size, when the library allocates itself); a call
 *    repeated at the same sizes only enqueues, so it can be captured in a
 *    HIP graph.  A captured graph keeps the addresses of the context's
 *    workspaces: it stays valid only while no later call on that context
 *    grows a workspace (a growing call frees the old one).  To rule that
 *    out, run the calls to be captured once, then dfacto_ctx_freeze(ctx, 1):
 *    from then on a call that would grow a workspace fails with
 *    DFACTO_E_INVALID instead.  Inputs must stay unmodified until the
 *    stream passes the call.
 *  - Every call returns a status; nothing aborts, throws or prints.  A HIP
 *    runtime failure is sticky: the context then returns DFACTO_E_DEVICE
 *    from every later call.  dfacto_last_error() describes the last failure.
 *  - Results are bitwise reproducible for a given tensor, R and dtype: no
 *    floating-point atomics are used and every reduction has a fixed order.
 *  - One context per host thread.  A built tensor is read-only and may be
 *    used from several contexts on the same device.
 */
#ifndef DFACTO_H
#define DFACTO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DFACTO_OK = 0,
    DFACTO_E_INVALID = 1,     /* bad argument: null pointer, mode, R, dims, dtype */
    DFACTO_E_RANGE = 2,       /* a coordinate is >= its dimension */
    DFACTO_E_NOMEM = 3,       /* a device allocation failed */
    DFACTO_E_DEVICE = 4,      /* HIP runtime error (sticky on the context) */
    DFACTO_E_NUMERIC = 5,     /* NaN or Inf among the tensor values */
    DFACTO_E_UNSUPPORTED = 6, /* sizes beyond the supported limits */
    DFACTO_E_AGAIN = 7        /* a served result is not ready yet */
} dfacto_status;

typedef enum { DFACTO_F32 = 0, DFACTO_BF16 = 1 } dfacto_dtype;

/* Limits.  Each dimension must be in [1, DFACTO_MAX_DIM]; nnz plus the
 * number of fiber headers must stay below 2^32 - 2^20; R in [1, DFACTO_MAX_R]. */
#define DFACTO_MAX_DIM ((int64_t)1 << 30)
#define DFACTO_MAX_R 256

typedef struct dfacto_ctx dfacto_ctx;       /* device, stream, workspace, sticky error */
typedef struct dfacto_tensor dfacto_tensor; /* the three flattenings, on the device */

/* ------------------------------------------------------------------ */
/* context                                                              */
/* ------------------------------------------------------------------ */

/* A caller's source of device memory, so that a framework's own caching
 * allocator can own what the library allocates.  alloc(bytes, stream, user)
 * returns device memory of `bytes` bytes usable on `stream` (a hipStream_t),
 * aligned to 256 bytes, or NULL when it cannot (the call then fails with
 * DFACTO_E_NOMEM).  free(ptr, stream, user) gives it back; `stream` is the
 * stream of the memory's last use, and the allocator must not hand the
 * memory out again before that stream's work up to the free has finished
 * (stream-ordered reuse, as hipFreeAsync).  Both are called only from the
 * thread that calls the library, during its calls (and dfacto_*_destroy). */
typedef struct dfacto_allocator {
    void *(*alloc)(size_t bytes, void *stream, void *user);
    void (*free)(void *ptr, void *stream, void *user);
    void *user;
} dfacto_allocator;

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the default stream).
 * alloc: NULL, and the library allocates itself (hipMalloc for tensors and
 * workspaces, stream-ordered hipMallocAsync for build temporaries); or the
 * caller's allocator, which then serves every device allocation made on the
 * context's behalf: the flattenings of the tensors it builds (which keep
 * the allocator and the context's stream of that time for their
 * dfacto_tensor_destroy), build temporaries, workspaces and group
 * workspaces.  The struct is copied; the functions and `user` must stay
 * valid until the context and everything built with it are destroyed.
 * Errors: DFACTO_E_INVALID (out NULL, device out of range, alloc given with
 * a NULL function), DFACTO_E_DEVICE (no HIP device). */
dfacto_status dfacto_ctx_create(int device, void *hip_stream, const dfacto_allocator *alloc,
                                dfacto_ctx **out);

/* Rebind the context to another stream of the same device. */
dfacto_status dfacto_ctx_set_stream(dfacto_ctx *ctx, void *hip_stream);

/* Wait until all work the context enqueued has finished. */
dfacto_status dfacto_ctx_synchronize(dfacto_ctx *ctx);

/* Freeze (on = 1) or unfreeze (0) the context's workspaces.  While frozen,
 * a call that needs a larger workspace than the context holds fails with
 * DFACTO_E_INVALID and enqueues nothing, so workspace addresses recorded in
 * a HIP graph stay valid.  Size the workspaces first by running each call
 * to be captured once at its largest sizes. */
dfacto_status dfacto_ctx_freeze(dfacto_ctx *ctx, int on);

/* Free the context and its workspace.  NULL is ignored. */
void dfacto_ctx_destroy(dfacto_ctx *ctx);

/* Message for the last failing call on `ctx` (owned by ctx, valid until
 * the next call).  Never NULL. */
const char *dfacto_last_error(const dfacto_ctx *ctx);

/* ------------------------------------------------------------------ */
/* tensor: the three fiber-compressed flattenings                       */
/* ------------------------------------------------------------------ */

/* Build the three flattenings of the tensor of size dims[0] x dims[1] x
 * dims[2] given in coordinate format (d_i[e], d_j[e], d_k[e]) -> d_val[e],
 * e < nnz, all four arrays on the device (u32 indices, FP32 values).
 *
 * Section 2.1, eq. (1) defines the flattenings X1 (I x JK), X2 (J x KI),
 * X3 (K x IJ); Section 3 stores (X2)^T with its all-zero rows removed and
 * the sparsity pattern of the matrices M^r precomputed (Lemmas 3 and 4).
 * Here mode n keeps the nonzeros sorted by (root, mid, leaf):
 *     mode 0: (i, k, j)   mode 1: (j, i, k)   mode 2: (k, j, i)
 * i.e. the products of Algorithm 4 (Appendix E).  A fiber is a maximal run
 * of equal (root, mid); only nonempty fibers and roots are stored.
 * Duplicate coordinates are summed (in input order).  nnz = 0 is valid.
 *
 * Errors: DFACTO_E_INVALID (null pointers with nnz > 0, dims outside
 * [1, DFACTO_MAX_DIM], nnz < 0), DFACTO_E_RANGE (a coordinate out of range),
 * DFACTO_E_NUMERIC (NaN/Inf value), DFACTO_E_UNSUPPORTED (too many
 * entries), DFACTO_E_NOMEM.  This call synchronizes the stream.  The COO
 * arrays are not retained.  *out is owned by the caller: free it with
 * dfacto_tensor_destroy. */
dfacto_status dfacto_build_flattenings(dfacto_ctx *ctx, const int64_t dims[3], int64_t nnz,
                                       const uint32_t *d_i, const uint32_t *d_j,
                                       const uint32_t *d_k, const float *d_val,
                                       dfacto_tensor **out);

/* Build flags.  The MTTKRP gathers one factor row per stored nonzero (its
 * leaf) and one per fiber (its mid), and most gathers of a skewed tensor
 * fall on few rows.  A relabeled build stores, in place of those indices,
 * each row's rank in the order of decreasing gather count (ties by index;
 * one order per gathered table and mode); the MTTKRP then reads the factors
 * through copies permuted into that order, where the most-gathered rows
 * share cache lines (rows shorter than a line: BF16 factors, small R).
 * The nonzeros' order, and so every result, is the same either way.
 * DFACTO_BUILD_RELABEL: relabel; DFACTO_BUILD_NO_RELABEL: plain indices;
 * neither (dfacto_build_flattenings): relabel from 2^23 nonzeros on when
 * there are at least 64 nonzeros per factor row (nnz >= 64 (I + J + K)):
 * each MTTKRP of a relabeled tensor first copies its two gathered factors
 * into rank order, which pays only when rows are gathered often.  Rows
 * shorter than 128 bytes are copied at a stride of the next power of two
 * columns (zero filled), so that none straddles two cache lines; the
 * MTTKRP then writes a padded output in a context workspace and narrows it
 * into the caller's R columns (workspace per call: the two copies plus
 * dims x stride x 4 bytes of output, three outputs for the GD gradient). */
#define DFACTO_BUILD_RELABEL 1
#define DFACTO_BUILD_NO_RELABEL 2

/* Default stream entries per MTTKRP work chunk (a chunk is the unit of work
 * of one lane group; it ends at the first header at or after a multiple of
 * the chunk length). */
#define DFACTO_CHUNK_DEFAULT 512

/* dfacto_build_flattenings with build flags (above) and the work-chunk
 * length: chunk_len stream entries per chunk, 0 for DFACTO_CHUNK_DEFAULT,
 * else in [256, 2^20].  Longer chunks mean fewer carries to fix up and
 * fewer, longer work items; shorter ones spread a small tensor over more
 * lanes.  A row split over chunks is summed from per-chunk partial sums, so
 * results of different chunk lengths agree up to FP32 rounding, not
 * bitwise.  Errors as dfacto_build_flattenings, and
 * DFACTO_E_INVALID for unknown or contradictory flags or a chunk length out
 * of range. */
dfacto_status dfacto_build_flattenings_ex(dfacto_ctx *ctx, const int64_t dims[3], int64_t nnz,
                                          const uint32_t *d_i, const uint32_t *d_j,
                                          const uint32_t *d_k, const float *d_val, int flags,
                                          int chunk_len, dfacto_tensor **out);

typedef struct {
    int64_t dims[3];
    int64_t nnz;        /* distinct nonzeros after merging duplicates */
    int64_t nfib[3];    /* nonempty fibers per mode: nnzc of the paper's flattening */
    int64_t nroot[3];   /* nonempty output rows per mode */
    int64_t nentry[3];  /* length of the per-mode stream (nonzeros + fiber headers) */
    int64_t nchunk[3];  /* work chunks per mode */
    double normsq;      /* ||X||^2 in FP64 */
    size_t bytes;       /* device bytes held by the tensor */
    int relabeled;      /* 1 when built with relabeled gathers */
    int chunk_len;      /* stream entries per work chunk (target) */
} dfacto_tensor_info;

dfacto_status dfacto_tensor_get_info(const dfacto_tensor *t, dfacto_tensor_info *info);

/* Copy mode `mode`'s flattening to host memory in CSR form, for inspection
 * and tests: h_root_id[nroot], h_root_ptr[nroot+1] (fiber offsets),
 * h_fib_mid[nfib], h_fib_ptr[nfib+1] (nonzero offsets), h_leaf[nnz],
 * h_val[nnz].  Sizes come from dfacto_tensor_get_info.  Synchronizes. */
dfacto_status dfacto_tensor_export(dfacto_ctx *ctx, const dfacto_tensor *t, int mode,
                                   uint32_t *h_root_id, int64_t *h_root_ptr,
                                   uint32_t *h_fib_mid, int64_t *h_fib_ptr,
                                   uint32_t *h_leaf, float *h_val);

/* The row order of a relabeled mode's gathered table, for inspection and
 * tests: h_order[r] = the factor row ranked r, in the order of decreasing
 * gather count (table 0: the leaf table, counting the nonzeros of each leaf
 * row; table 1: the mid table, counting the fiber segment headers of each
 * mid row; ties by row index).  h_order holds dims[leaf] or dims[mid]
 * entries (leaf of mode n is mode (n+1) mod 3, mid is (n+2) mod 3).
 * Errors: DFACTO_E_INVALID for a NULL argument, a bad mode or table, or a
 * tensor built without relabeling.  Synchronizes. */
dfacto_status dfacto_tensor_gather_order(dfacto_ctx *ctx, const dfacto_tensor *t, int mode,
                                         int table, uint32_t *h_order);

/* Free a tensor (waits for the device).  NULL is ignored. */
void dfacto_tensor_destroy(dfacto_tensor *t);

/* ------------------------------------------------------------------ */
/* hot path                                                             */
/* ------------------------------------------------------------------ */

/* MTTKRP of `mode`: d_out (dims[mode] x R, FP32, overwritten) =
 *     mode 0: X1 (C kr B)    mode 1: X2 (A kr C)    mode 2: X3 (B kr A)
 * with d_F = {A, B, C} (d_F[mode] is not read and may be NULL).
 * Computed as Algorithm 1 for all R columns at once: per fiber the partial
 * P = sum_leaf x * F_leaf[leaf, :] (the values of M^r, Lemma 2), then per
 * output row the sum over its fibers of P * F_mid[mid, :]; FP32
 * accumulation, factor rows widened from the storage dtype.  Rows with no
 * nonzeros are written as zeros.  Enqueue only. */
dfacto_status dfacto_mttkrp(dfacto_ctx *ctx, const dfacto_tensor *t, int mode, int R,
                            dfacto_dtype dtype, const void *const d_F[3], float *d_out);

/* dfacto_mttkrp for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same computation and kernels, bitwise the same result, with the
 * call's buffers -- the carries of output rows split over work chunks and,
 * for a relabeled tensor, the factor tables permuted into rank order -- in
 * a fixed device array of 64 MiB that the library holds on every GPU it
 * runs on until the process ends.  It calls no allocator and takes no
 * workspace of the context.  Every call on a GPU shares that GPU's array:
 * calls that overlap on one GPU (other streams, other threads) race, and
 * must be ordered by the caller.  Arguments as dfacto_mttkrp.  Errors as
 * there, and DFACTO_E_UNSUPPORTED when the call needs more than the array
 * holds (nchunk x R x 4 bytes of carries, plus for a relabeled tensor the
 * two gathered factors' rows), DFACTO_E_INVALID for a tensor built on
 * another device. */
dfacto_status dfacto_mttkrp_noalloc(dfacto_ctx *ctx, const dfacto_tensor *t, int mode, int R,
                                    dfacto_dtype dtype, const void *const d_F[3], float *d_out);

/* One CP-ALS iteration (Algorithm 2 / Algorithm 4), in place on
 * d_F = {A, B, C}, modes updated in the order 0, 1, 2, each with the
 * factors already updated:
 *     M_n = MTTKRP(n);  H = (F_p^T F_p) * (F_q^T F_q) + reg I;
 *     F_n = M_n H^{-1}  (FP64 Cholesky; Moore-Penrose pseudo-inverse when
 *     H is numerically singular);  lambda_r = ||F_n[:, r]||_2;
 *     F_n[:, r] /= lambda_r (zero columns stay zero, lambda_r = 0).
 * reg is the ridge parameter of the regularized update (Appendix B),
 * reg >= 0.  On return d_lambda (R doubles) holds the weights from the
 * mode-2 normalization and *d_fit (one double) the fit
 *     1 - ||X - [[lambda; A, B, C]]|| / ||X||   (0 when ||X|| = 0).
 * With DFACTO_BF16 the factors are stored rounded (to FP32, then BF16,
 * nearest-even), and each later mode's Gram is formed from the stored
 * factor, so the normal equations match what the MTTKRPs read.
 * Enqueue only (no host synchronization); d_lambda and d_fit are device
 * pointers. */
dfacto_status dfacto_als_iter(dfacto_ctx *ctx, const dfacto_tensor *t, int R,
                              dfacto_dtype dtype, double reg, void *const d_F[3],
                              double *d_lambda, double *d_fit);

/* GD gradient (Appendix C; Algorithm 3) at the point d_F = {A, B, C} with
 * unit weights, all three gradients at the same point:
 *     d_G[n] = -MTTKRP(n) + F_n ((F_p^T F_p) * (F_q^T F_q) + reg I)
 * (FP32, dims[n] x R each) and *d_f (device double) the objective
 *     1/2 ||X - [[A, B, C]]||^2 + reg/2 (||A||^2 + ||B||^2 + ||C||^2),
 * summed over every (i, j, k).  Enqueue only. */
dfacto_status dfacto_gd_grad(dfacto_ctx *ctx, const dfacto_tensor *t, int R,
                             dfacto_dtype dtype, double reg, const void *const d_F[3],
                             float *const d_G[3], double *d_f);

/* ------------------------------------------------------------------ */
/* grouped CP-ALS (many independent solves at once)                     */
/* ------------------------------------------------------------------ */

/* A group runs CP-ALS iterations (the same iteration as dfacto_als_iter) for
 * n independent tensors together: every step of an iteration is one kernel
 * launch per kernel class for all members (the MTTKRP as a persistent grid
 * over a work list of (member, chunk group) items), so small tensors do not
 * pay one launch each.  Per member the results are bitwise those of
 * dfacto_als_iter on the same inputs.
 *
 * Members: tensors[t] (built on ctx's device; they must outlive the group),
 * ranks[t] in {4, 8, 12, 16, 32, 48, 64}, one storage dtype for all, factors
 * d_F[3 t + m] (row-major dims[m] x ranks[t], device, 16-byte aligned,
 * updated in place), d_lambda[t] (ranks[t] doubles, device) and d_fit[t]
 * (device double).  All pointers are caller-owned and must stay valid while
 * the group lives.  The group allocates its own workspace and tables
 * (reported by dfacto_group_get_info; from ctx's memory source, the caller's
 * allocator when one was given) and uses its own HIP stream, ordered after
 * ctx's stream by events at each call.
 *
 * flags: DFACTO_GROUP_GRAPH captures one iteration as a HIP graph on the
 * first dfacto_group_als call and replays it; DFACTO_GROUP_TUNE times each
 * MTTKRP launch at creation in several forms -- persistent grid sizes of 2
 * to 32 workgroups per CU, other factor columns per lane (fewer, or eight
 * for BF16 ranks that are multiples of 8) with the lanes per group to
 * match, 1, 2 or 4 work chunks per lane group -- and keeps the fastest
 * (results do not depend on the choice); DFACTO_GROUP_CTX_STREAM
 * launches on the creating context's stream instead of a stream of the
 * group's own (cheaper to create and free; later calls must pass a context
 * with that same stream).  Creation enqueues the upload and device-side
 * assembly of the group's tables on its stream and returns without waiting
 * (DFACTO_GROUP_TUNE waits for its timings); E_UNSUPPORTED for a rank
 * outside the list above. */
#define DFACTO_GROUP_GRAPH 1
#define DFACTO_GROUP_TUNE 2
#define DFACTO_GROUP_CTX_STREAM 4
/* The caller does not write the members' factors between dfacto_group_als
 * calls (only the group's iterations change them).  With BF16 storage an
 * iteration opens with the Grams of the stored B and C, which the previous
 * iteration has just formed for the same factors; they are reused after
 * the first iteration of every call anyway, and with this flag also across
 * calls.  Results are the same bitwise. */
#define DFACTO_GROUP_OWN_FACTORS 8

typedef struct dfacto_group dfacto_group;

typedef struct {
    int members;
    int launches_per_iter;  /* kernel launches in one iteration */
    size_t bytes;           /* device workspace and tables owned by the group */
    int graph;              /* 1 when iterations replay a captured graph */
    int mttkrp_classes;     /* MTTKRP launches per iteration */
    int mttkrp_grid[16];    /* their persistent grid sizes (first 16) */
    int mttkrp_cpl[16];     /* factor columns per lane */
    int mttkrp_lanes[16];   /* lanes per group */
    int mttkrp_chunks_per_group[16];  /* work chunks each lane group takes in turn */
    int mttkrp_forms[16];   /* launch forms considered (1 without tuning) */
} dfacto_group_info;

dfacto_status dfacto_group_create(dfacto_ctx *ctx, int n, const dfacto_tensor *const *tensors,
                                  const int *ranks, dfacto_dtype dtype, double reg,
                                  void *const *d_F, double *const *d_lambda, double *d_fit,
                                  int flags, dfacto_group **out);

/* Enqueue `iters` CP-ALS iterations of every member (no host
 * synchronization; the fits are written to d_fit each iteration). */
dfacto_status dfacto_group_als(dfacto_ctx *ctx, dfacto_group *g, int iters);

dfacto_status dfacto_group_get_info(const dfacto_group *g, dfacto_group_info *info);

/* Choose MTTKRP launch class `cls`'s form explicitly: form index `form`
 * among the mttkrp_forms[cls] forms (form 0 is the default; a group created
 * without DFACTO_GROUP_TUNE has only that one) and persistent grid size
 * `grid` (>= 1 workgroups).  For callers that replay a choice recorded from
 * an earlier tuning, and for tests of every form; results do not depend on
 * it.  A captured iteration graph is dropped and captured again at the
 * next dfacto_group_als.  Must not overlap a dfacto_group_als call on the
 * same group.  Errors: DFACTO_E_INVALID (NULL group, index or grid out of
 * range). */
dfacto_status dfacto_group_set_form(dfacto_group *g, int cls, int form, int grid);

/* Free the group (waits for its stream).  NULL is ignored. */
void dfacto_group_destroy(dfacto_group *g);

/* ------------------------------------------------------------------ */
/* served solves with continuous batching                               */
/* ------------------------------------------------------------------ */

/* A server runs CP-ALS solves submitted at any time on one device.  It owns
 * a device-memory budget, a worker thread, two builder threads (each with
 * its own HIP stream) and a delivery thread.  The builders admit queued
 * requests in arrival order while a slot is free and their device footprint
 * fits the budget (the three flattenings, each at most about the size of
 * the COO tensor, plus factors and workspace, plus the transient memory of
 * one build) and build them while the worker iterates.  At every iteration
 * boundary the worker attaches the built requests, runs one grouped CP-ALS
 * iteration of every active request, and retires the requests that met
 * their stopping rule; the delivery thread copies their results to the host
 * and frees their memory for the queue.  A request's results do not depend on which others run with it: they are
 * bitwise those of dfacto_als_iter repeated on it alone.
 *
 * hbm_budget: device bytes the server may hold (0 = 90% of the free memory
 * at creation); max_slots: most requests active at once (>= 1).
 *
 * Measured on MI355X: a server created in a process where another server
 * has already run (and been destroyed) serves 20-35% fewer solves per
 * second than the first one did; keep one server for the life of a process
 * where throughput matters. */
typedef struct dfacto_server dfacto_server;

typedef struct {
    /* input, host memory, owned by the caller until the request is done */
    int64_t dims[3];
    int64_t nnz;
    const uint32_t *i, *j, *k; /* coordinates (as for dfacto_build_flattenings) */
    const float *val;
    int R;                     /* in {4, 8, 12, 16, 32, 48, 64} */
    dfacto_dtype dtype;        /* factor storage on the device */
    double reg;                /* ridge parameter (>= 0) */
    const float *init[3];      /* initial factors, dims[m] x R, FP32 */
    double tol;                /* stop when |fit - previous fit| < tol ... */
    int max_iters;             /* ... or after max_iters iterations (>= 1) */
    /* output, host memory, owned by the caller (may be NULL) */
    float *out_F[3];           /* final factors, dims[m] x R, FP32 */
    double *out_lambda;        /* final weights, R */
} dfacto_request;

typedef struct {
    int done;                  /* 1 once finished */
    dfacto_status status;      /* OK, or the error that ended the request */
    double fit;                /* fit after the last iteration */
    int iters;                 /* iterations run */
    double t_submit, t_admit, t_done; /* seconds on the server's clock */
} dfacto_request_status;

typedef struct {
    int64_t pending, running, finished;
    int peak_active;           /* most requests active at one time */
    int64_t iterations;        /* iteration boundaries run */
    size_t budget;
    /* wall time, seconds: builders uploading, building and initializing
     * admitted requests (summed over the builders), of that the flattening
     * builds; worker (re)building groups and running iterations (incl.
     * reading the fits); delivery thread copying results out */
    double t_admit, t_build, t_groups, t_iterate, t_deliver;
} dfacto_server_stats;

dfacto_status dfacto_server_create(int device, size_t hbm_budget, int max_slots,
                                   dfacto_server **out);

/* Queue a request (copied; its host arrays are read at admission and the
 * outputs written at completion).  *id identifies it.  E_INVALID for bad
 * arguments, E_UNSUPPORTED for a rank outside the list above. */
dfacto_status dfacto_server_submit(dfacto_server *srv, const dfacto_request *req, int64_t *id);

/* OK with the final status once the request is done, E_AGAIN before. */
dfacto_status dfacto_server_poll(dfacto_server *srv, int64_t id, dfacto_request_status *st);

/* Block until the request is done. */
dfacto_status dfacto_server_wait(dfacto_server *srv, int64_t id, dfacto_request_status *st);

dfacto_status dfacto_server_get_stats(dfacto_server *srv, dfacto_server_stats *out);

/* Finish every submitted request, then free the server.  NULL is ignored. */
void dfacto_server_destroy(dfacto_server *srv);

/* ------------------------------------------------------------------ */
/* measurement                                                          */
/* ------------------------------------------------------------------ */

/* ------------------------------------------------------------------ */
/* joint matrix completion and tensor factorization                     */
/* ------------------------------------------------------------------ */

/* The joint model of the paper's section on joint matrix completion and
 * tensor factorization: a ratings matrix Y (users x items, observed entries
 * only) shares the user factor A and the item factor B with a
 * users x items x words tensor X (factor C):
 *   f = 1/2 sum_{(i,j) observed} (y_ij - a_i . b_j)^2
 *       + mu 1/2 sum_{i,j,k} (x_ijk - [[A,B,C]]_ijk)^2
 *       + lam 1/2 (||A||^2 + ||B||^2 + ||C||^2)
 * (the tensor sum runs over every cell, as in dfacto_gd_grad).
 *
 * dfacto_build_ratings builds Y from n device COO entries (d_i[e], d_j[e])
 * -> d_y[e] (u32 indices below dims[0] x dims[1], FP32 values; duplicates
 * summed) as a dims[0] x dims[1] x 1 tensor (so its MTTKRPs with a row of
 * ones as third factor are Y B and Y^T A, computed by the DFacTo kernels)
 * plus per-row entry ranges for the ALS rows.  Errors and ownership as
 * dfacto_build_flattenings; synchronizes the stream. */
dfacto_status dfacto_build_ratings(dfacto_ctx *ctx, const int64_t dims[2], int64_t n,
                                   const uint32_t *d_i, const uint32_t *d_j, const float *d_y,
                                   dfacto_tensor **out);

/* Gradients of the joint f at one point (the paper's per-row gradient
 * equation, all rows, all three factors) and f:
 *   dA = -sum_j (y_ij - a_i.b_j) b_j + mu (-M_0 + A (B^T B * C^T C)) + lam A
 *   dB = -sum_i (y_ij - a_i.b_j) a_i + mu (-M_1 + B (A^T A * C^T C)) + lam B
 *   dC =                                mu (-M_2 + C (A^T A * B^T B)) + lam C
 * The ratings terms are residual MTTKRPs of Y (FP32 accumulation); the
 * ratings part of f is formed as 1/2 (||Y||^2 - <A, Y B> - <A, residual B>)
 * in FP64.  X and Y must share dims[0] and dims[1]; mu, lam >= 0.  Factor
 * and gradient layouts, dtypes and errors as dfacto_gd_grad; Y not built by
 * dfacto_build_ratings or of the wrong shape: DFACTO_E_INVALID.  Enqueues
 * only. */
dfacto_status dfacto_joint_grad(dfacto_ctx *ctx, const dfacto_tensor *X, const dfacto_tensor *Y,
                                int R, dfacto_dtype dtype, double mu, double lam,
                                const void *const d_F[3], float *const d_G[3], double *d_f);

/* One ALS iteration of the joint model, A, B, C in order, each row set to
 * the minimizer with the other factors fixed (the paper's closed form):
 *   a_i = (sum_j y_ij b_j + mu M_0[i]) (sum_j b_j^T b_j + mu B^T B * C^T C + lam I)^-1
 * over the items j rated by user i, likewise b_j over the users who rated j,
 * and c_k = mu M_2[k] (mu A^T A * B^T B + lam I)^-1.  Each user's and item's
 * R x R system is formed and inverted in FP64 by one wavefront; factors are
 * updated in place in their dtype (no column normalization).  Needs lam > 0
 * (every system is then positive definite) and R <= 32
 * (DFACTO_E_UNSUPPORTED above); DFACTO_E_NUMERIC if a system still fails
 * the positive-definiteness test.  Synchronizes the stream (the test's
 * flag is read back). */
dfacto_status dfacto_joint_als_iter(dfacto_ctx *ctx, const dfacto_tensor *X,
                                    const dfacto_tensor *Y, int R, dfacto_dtype dtype, double mu,
                                    double lam, void *const d_F[3]);

/* One full GD iteration (Algorithm 5 of Appendix E; Algorithm 3 of
 * Appendix C): the three gradients at the same point (as dfacto_gd_grad,
 * written to d_G), then a backtracking line search, then the simultaneous
 * update of the three factors.  The paper names a backtracking line search
 * without giving its rule; this one is Armijo's: trial steps
 * alpha = alpha0 * shrink^t for t = 0 .. max_trials - 1 form the trial
 * factors F_m - alpha grad_m (in FP64 from the stored factor and the FP32
 * gradient, stored in the factor dtype), and the first trial with
 *     f(trial) <= f(F) - c * alpha * (||grad_A||^2 + ||grad_B||^2 + ||grad_C||^2)
 * replaces the factors.  f(trial) is computed as in dfacto_gd_grad (three
 * Grams, the mode-0 MTTKRP of the trial point, FP64 reductions).  If no
 * trial passes, the factors are left unchanged and info->accepted = 0.
 *
 * d_F: in/out factors (layout and alignment as dfacto_gd_grad); d_G: the
 * gradients at the input point (out); ls: host struct; info: host struct,
 * filled on return.  The trial factors live in a context workspace
 * (sum of the factor sizes plus one dims[0] x R FP32 buffer).  Synchronizes
 * the stream once per trial (the test needs f on the host).  Errors: as
 * dfacto_gd_grad, plus DFACTO_E_INVALID for a NULL ls or info, alpha0 <= 0
 * or not finite, shrink or c outside (0, 1), max_trials outside [1, 1000]. */
typedef struct {
    double alpha0;   /* first trial step, > 0 */
    double shrink;   /* step factor after a rejected trial, in (0, 1) */
    double c;        /* sufficient-decrease constant, in (0, 1) */
    int max_trials;  /* trials at most, in [1, 1000] */
} dfacto_linesearch;

typedef struct {
    double f0;       /* objective at the input factors */
    double f;        /* objective at the returned factors */
    double gnorm2;   /* squared norm of the gradient (all three factors) */
    double alpha;    /* step taken, 0 when no trial passed */
    int trials;      /* trials evaluated */
    int accepted;    /* 1 if the factors were updated */
} dfacto_gd_step_info;

dfacto_status dfacto_gd_step(dfacto_ctx *ctx, const dfacto_tensor *t, int R, dfacto_dtype dtype,
                             double reg, void *const d_F[3], float *const d_G[3],
                             const dfacto_linesearch *ls, dfacto_gd_step_info *info);

/* Turn kernel timing on (1) or off (0) for `ctx`.  While on, every MTTKRP
 * launch (also those inside dfacto_als_iter and dfacto_gd_grad) records a
 * pair of HIP events on the context's stream around its main kernel, and
 * adds the launch's algorithmic byte count (Section 3.2 work model:
 * 8 B per stored nonzero, 8 B per fiber, 8 B per nonempty row, the output
 * rows and one read of each factor that is gathered).  Turning it on
 * clears earlier records. */
dfacto_status dfacto_profile_enable(dfacto_ctx *ctx, int on);

/* Synchronize and report what was recorded since timing was enabled (or
 * last read): *launches main-kernel launches, *ms their summed duration,
 * *bytes their summed algorithmic bytes, *flops their summed
 * 2 R (nnz + nfib) flops.  Clears the records.  Any pointer may be NULL. */
dfacto_status dfacto_profile_read(dfacto_ctx *ctx, int64_t *launches, double *ms, double *bytes,
                                  double *flops);

/* Measurement of the MTTKRP's memory-request ceiling (Section 3.2: the
 * product is a scan of the mode's flattening with one factor-row gather per
 * stored nonzero and per fiber).  Runs the main MTTKRP kernel's memory
 * requests for `mode` -- the same work chunks, lane groups, batches and row
 * loads -- with the arithmetic replaced by a plain sum of each gathered row.
 * pattern 0: each entry gathers its own row (the MTTKRP's exact request
 * sequence); 1: a row drawn uniformly at random from the same factor (leaf
 * factor for a nonzero, mid factor for a header); 2: a row among that
 * factor's first 4096; 3: no gathers, the flattening is only read; 4: a row
 * among the factor's first 32; 5: a row of a 128-row table held in LDS
 * (R <= 64); 6-9 gather leaf rows (a header's mid index taken modulo the
 * leaf rows) with buffer loads: 6 every load out of range (no memory
 * request), 7 the entry's own row, 8 half of the entries (by a hash bit)
 * from the LDS table and half their own rows, split by a branch, 9 the same
 * split without a branch (an out-of-range load beside an LDS load).
 * d_F as for dfacto_mttkrp (only R <= 64 x the kernel's columns per lane);
 * d_sink: device buffer of at least 64 x (work chunks of the mode) floats,
 * 16-byte aligned, overwritten with meaningless sums.  With timing on
 * (dfacto_profile_enable) the launch is recorded like an MTTKRP's main
 * kernel, without bytes.  Errors: DFACTO_E_INVALID (arguments),
 * DFACTO_E_UNSUPPORTED (R too large for one column block). */
dfacto_status dfacto_gather_probe(dfacto_ctx *ctx, const dfacto_tensor *t, int mode, int R,
                                  dfacto_dtype dtype, const void *const d_F[3], int pattern,
                                  float *d_sink);

#ifdef __cplusplus
}
#endif

#endif /* DFACTO_H */
