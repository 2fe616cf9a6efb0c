// internal.hpp -- shared declarations of the DFacTo HIP library (not public).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "dfacto.h"

namespace dfacto {

// ---------------------------------------------------------------------------
// Per-mode stream layout (one 8-byte entry per nonzero or fiber header)
//
//   nonzero : x = leaf index,                      y = float bits of the value
//   header  : x = HDR | (ROOT if a root starts) | mid index,   y = output row
//
// A header opens a fiber segment: the nonzeros that follow, up to the next
// header, share (root, mid).  Fibers longer than kFiberCap nonzeros are cut
// into segments, each with its own header (same root and mid, no ROOT bit),
// so that work chunks -- which always start at a header -- stay balanced.
// ---------------------------------------------------------------------------
constexpr uint32_t kHdrBit = 0x80000000u;
constexpr uint32_t kRootBit = 0x40000000u;
constexpr uint32_t kIdxMask = 0x3FFFFFFFu;
constexpr int kFiberCap = 128;     // max nonzeros per fiber segment
constexpr int kStreamPad = 64;     // sentinel entries after the stream end

struct ModeData {
    int root = 0, mid = 0, leaf = 0;   // coordinate axes (0 = i, 1 = j, 2 = k)
    uint2 *stream = nullptr;           // nentry + kStreamPad entries
    int64_t nentry = 0;
    int64_t nfib = 0, nroot = 0;
    uint32_t *empty_rows = nullptr;    // output rows with no nonzeros
    int64_t nempty = 0;
    // work chunks: chunk c covers stream entries [chunk_start[c], chunk_start[c+1])
    uint32_t *chunk_start = nullptr;   // nchunk + 1 entries
    int64_t nchunk = 0;
    int chunk_len = 0;                 // target entries per chunk
    // Output rows whose nonzeros span several chunks ("runs"): the chunk that
    // starts the row writes it, chunks c0 .. c0+n-1 write carries.  Runs of at
    // most kShortRun carries are summed by one lane group, longer runs by a
    // whole workgroup.  Each list holds (row, c0, n) triplets.
    uint32_t *runs_short = nullptr;
    int64_t nruns_short = 0;
    uint32_t *runs_long = nullptr;
    int64_t nruns_long = 0;
    // host copies of the run lists (the sources of their uploads)
    std::vector<uint32_t> runs_short_host, runs_long_host;
    // Relabeled gathers (null when the stream holds the original indices):
    // the stream's leaf and mid indices are ranks in the order of decreasing
    // gather count (nonzeros per leaf row, fiber headers per mid row; ties
    // by index), so row r of a gathered table is factor row perm_*[r] and
    // the most-gathered rows are the first ones.
    uint32_t *perm_leaf = nullptr, *perm_mid = nullptr;
};
// dfacto_build_flattenings relabels the gathers of tensors from this size on,
// when they hold at least kRelabelPerRow nonzeros per factor row (the copies
// into rank order cost a pass over the gathered factors per MTTKRP, which
// the shared lines repay only when each row is gathered often)
constexpr int64_t kRelabelMinNnz = (int64_t)1 << 23;
constexpr int64_t kRelabelPerRow = 64;

constexpr int kShortRun = 16;

// MTTKRP kernel shape: CPL consecutive columns per lane, lane groups of G
// lanes, NCH column blocks per lane.
struct MttkrpShape {
    int cpl, g, nch;
};

// Arguments of the dense steps per tensor, for grouped launches.
struct GramJob {
    const void *F;
    int64_t rows;
    int R;
    uint32_t nblk;  // partial blocks (gram_plan)
    double *part;   // nblk x R x R partial sums
    double *G;      // R x R result
};
struct SolveJob {
    int R;
    double reg;
    const double *Gp, *Gq;
    double *Hinv, *scratch;
    int *flag;
};
struct LambdaJob {
    int R, mode;
    const double *Hinv, *MtM;
    double *Gn, *W, *lambda;
    const double *GA, *GB;
    double normsq;
    double *fit, *scratch;
};
// The fit from a stored (rounded) last factor, per tensor.
struct FitJob {
    const void *F;    // stored mode-2 factor, rows x R
    const float *M;   // its MTTKRP
    int64_t rows;
    int R;
    uint32_t nblk;    // partial blocks (fit_blocks)
    const double *lambda, *GA, *GB, *GC;
    double normsq;
    double *part;     // nblk partial sums
    double *fit;
};
struct RowmapJob {
    const float *M;
    int64_t rows;
    const double *W;
    void *F;
    uint32_t nblk;
};
struct GramPlan {
    int nt = 0, nblk = 0;
    bool vec = false;
};
struct RowmapPlan {
    enum { kMfma = 0, kTiled = 1, kGeneric = 2 };
    int kind = kGeneric;
    uint32_t nblk = 0;
};

// Per-(tensor, mode) arguments of a grouped MTTKRP and its fix-ups.
struct GroupMttkrp {
    const uint2 *stream;
    const uint32_t *chunk_start;
    uint32_t nchunk;
    int R;
    const void *Fleaf, *Fmid;
    float *out, *carry;
};

// stream-ordered allocation from `pool`, or from the device default pool
inline hipError_t stream_alloc(void **p, size_t bytes, hipStream_t s, hipMemPool_t pool) {
    return pool ? hipMallocFromPoolAsync(p, bytes, pool, s) : hipMallocAsync(p, bytes, s);
}

// Where device memory made on a context's behalf comes from: the caller's
// callbacks when user.alloc is set, else stream-ordered allocation from
// `pool` (null: the device's default pool).  Every free names the stream the
// memory was last used on, so its reuse is ordered after that stream's work.
struct Arena;

struct DevMem {
    dfacto_allocator user{nullptr, nullptr, nullptr};
    hipMemPool_t pool = nullptr;
    // a build's bump allocator for its temporaries (set while a build runs)
    Arena *arena = nullptr;
    bool has_user() const { return user.alloc != nullptr; }
    hipError_t alloc(void **p, size_t bytes, hipStream_t s) const {
        if (has_user()) {
            *p = user.alloc(bytes, (void *)s, user.user);
            return *p ? hipSuccess : hipErrorOutOfMemory;
        }
        return stream_alloc(p, bytes, s, pool);
    }
    void free(void *p, hipStream_t s) const {
        if (!p) return;
        if (has_user()) user.free(p, (void *)s, user.user);
        else (void)hipFreeAsync(p, s);
    }
};

// Temporaries of one build: allocations up to kMaxTake bytes are carved
// from a few large chunks (each from the build's memory source) and all
// given back when the build ends, instead of one allocation and one free
// per temporary (a small build makes about eighty; each costs 10-30 us of
// host time in the runtime, several times the build's kernel time).
// Freed in stream order on the build's stream.
struct Arena {
    static constexpr size_t kMaxTake = (size_t)16 << 20;
    static constexpr size_t kFirstChunk = (size_t)16 << 20;
    hipStream_t s;
    DevMem mem;  // the chunks' source (no arena)
    std::vector<std::pair<char *, size_t>> chunks;
    char *cur = nullptr;
    size_t left = 0, next = kFirstChunk;
    Arena(hipStream_t st, const DevMem &m) : s(st), mem(m) { mem.arena = nullptr; }
    Arena(const Arena &) = delete;
    Arena &operator=(const Arena &) = delete;
    ~Arena() {
        for (auto &c : chunks) mem.free(c.first, s);
    }
    // nullptr: too large for the arena, or no device memory for a chunk
    void *take(size_t bytes) {
        bytes = (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
        if (bytes > kMaxTake) return nullptr;
        if (bytes > left) {
            const size_t c = std::max(bytes, next);
            void *p = nullptr;
            if (mem.alloc(&p, c, s) != hipSuccess) {
                (void)hipGetLastError();
                return nullptr;
            }
            chunks.push_back({(char *)p, c});
            cur = (char *)p;
            left = c;
            next = std::min<size_t>(2 * c, (size_t)1 << 30);
        }
        void *r = cur;
        cur += bytes;
        left -= bytes;
        return r;
    }
    bool owns(const void *p) const {
        for (const auto &c : chunks)
            if ((const char *)p >= c.first && (const char *)p < c.first + c.second) return true;
        return false;
    }
};

}  // namespace dfacto

struct dfacto_tensor {
    int device = 0;
    // when set, the tensor's memory is stream-ordered (from `mem`, on this
    // stream) and freeing it does not wait for unrelated device work;
    // otherwise it comes from hipMalloc
    hipStream_t alloc_stream = nullptr;
    dfacto::DevMem mem;
    int64_t dims[3] = {0, 0, 0};
    int64_t nnz = 0;
    double normsq = 0.0;
    bool relabel = false;  // build the streams with relabeled gathers
    int chunk_len = DFACTO_CHUNK_DEFAULT;  // target stream entries per work chunk
    size_t bytes = 0;
    dfacto::ModeData mode[3];
    std::vector<void *> allocations;
    char *slab = nullptr;  // the current slab of small arrays (build.hip)
    size_t slab_left = 0;
    // ratings matrix of the joint model (dims[2] == 1, built by
    // dfacto_build_ratings): per output row of modes 0 and 1, the range
    // [x, y) of its entries in that mode's stream ((0, 0) for an empty row)
    bool ratings = false;
    uint2 *row_range[2] = {nullptr, nullptr};
    // rows of more than kJointSeg entries, split into segments: seg_range[m]
    // (begin, end) per segment, heavy[m] (row, first segment, segments, 0)
    uint2 *seg_range[2] = {nullptr, nullptr};
    uint4 *heavy[2] = {nullptr, nullptr};
    int64_t nseg[2] = {0, 0}, nheavy[2] = {0, 0};
};

struct dfacto_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    // source of the device memory made on this context's behalf
    dfacto::DevMem mem;
    // a second stream for work that overlaps the main stream's (created on
    // first use), joined back by events
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_step = nullptr;
    int num_cu = 0;
    bool sticky = false;
    std::string err;
    // growable device workspace, one slot per purpose (Gram partial sums: one
    // slot per stream, so that Grams on the two streams may overlap)
    enum Slot {
        kM = 0, kCarry, kPartial, kPartialSide, kSmall, kTrial, kJoint, kPerm, kPadOut, kNumSlots
    };
    void *ws[kNumSlots] = {};
    size_t ws_size[kNumSlots] = {};
    bool frozen = false;  // dfacto_ctx_freeze: workspaces may not grow
    // build temporaries without a caller's memory source (created on the
    // first build; empty between builds)
    hipMemPool_t build_pool = nullptr;
    // kernel timing (dfacto_profile_*)
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;  // created on demand, reused
    size_t ev_used = 0;                // events handed out since the last read
    double prof_bytes = 0.0, prof_flops = 0.0;
};

namespace dfacto {

// Error plumbing: every entry point returns a status; HIP failures become
// sticky DFACTO_E_DEVICE on the context.
struct Error {
    dfacto_status code;
    std::string msg;
};

dfacto_status fail(dfacto_ctx *ctx, dfacto_status code, const std::string &msg);

// Pointers into device (global) memory.  Loads and stores through them are
// global instructions.  Through a plain pointer whose origin the compiler
// cannot see -- one read from a descriptor in memory, as in the grouped
// kernels -- they would be flat instructions, which count against the LDS
// counter as well, so every wait for an LDS result (the stream entries
// shared by ds_swizzle) would also wait for every gather in flight.
#define DF_GLOBAL __attribute__((address_space(1)))
// plain vector types for loads through such pointers (the HIP vector
// types cannot be copied out of a qualified address space)
typedef float df_f2 __attribute__((ext_vector_type(2)));
typedef float df_f4 __attribute__((ext_vector_type(4)));
typedef unsigned int df_u2 __attribute__((ext_vector_type(2)));
typedef unsigned int df_u4 __attribute__((ext_vector_type(4)));
template <typename T>
__device__ __forceinline__ const DF_GLOBAL T *gptr(const T *p) {
    return (const DF_GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ DF_GLOBAL T *gptr(T *p) {
    return (DF_GLOBAL T *)p;
}

void hip_check(hipError_t e, const char *what);  // throws Error on failure
#define DF_HIP(call) ::dfacto::hip_check((call), #call)
// after kernel launches: a launch error names the launching function
#define DF_LAUNCHED() ::dfacto::hip_check(hipGetLastError(), __func__)

void *ws_get(dfacto_ctx *ctx, dfacto_ctx::Slot slot, size_t bytes);

// Record one profiling event on the context stream (no-op when off).
void prof_mark(dfacto_ctx *ctx);

// ---------------------------------------------------------------------------
// kernels and launchers (implemented in the .hip files)
// ---------------------------------------------------------------------------

// device-wide primitives (build.hip)
// (temporaries from mem, the device default pool when null)
void scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t n, hipStream_t s,
                        const DevMem *mem = nullptr);

// builder (build.hip): fills t (allocates its arrays).  Synchronizes.
// dfacto_build_flattenings with stream-ordered tensor memory on ctx's stream
dfacto_status build_flattenings_async_alloc(dfacto_ctx *ctx, const int64_t dims[3], int64_t nnz,
                                            const uint32_t *d_i, const uint32_t *d_j,
                                            const uint32_t *d_k, const float *d_val,
                                            dfacto_tensor **out);
// per-row entry ranges of modes 0 and 1 (the joint model's ratings matrix)
void build_row_ranges(dfacto_ctx *ctx, dfacto_tensor *t);
void build_tensor(dfacto_ctx *ctx, dfacto_tensor *t, const uint32_t *d_i, const uint32_t *d_j,
                  const uint32_t *d_k, const float *d_val);

// MTTKRP (mttkrp.hip)
// Device bytes of the permuted copies a relabeled tensor's MTTKRPs gather
// from (0 when not relabeled), the largest over the modes.
size_t perm_bytes(const dfacto_tensor *t, int R, dfacto_dtype dtype);
// A relabeled mode's permuted tables in `buf` (perm_bytes): their places,
// and the launches that fill them from the factors (on ctx's stream).
void relabeled_tables(const dfacto_tensor *t, int mode, int R, dfacto_dtype dtype, void *buf,
                      const void **leaf, const void **mid);
void launch_relabeled_tables(dfacto_ctx *ctx, const dfacto_tensor *t, int mode, int R,
                             dfacto_dtype dtype, const void *Fleaf, const void *Fmid, void *buf);
void launch_mttkrp(dfacto_ctx *ctx, const dfacto_tensor *t, int mode, int R, dfacto_dtype dtype,
                   const void *Fleaf, const void *Fmid, float *out);
// The same with the carries in `carry` (nchunk x R floats of the caller's)
// and the carry fix-ups on stream `fix`, after `ev` recorded on ctx's stream
// behind the main kernel: `out` is complete in stream order on `fix`.
void launch_mttkrp_split(dfacto_ctx *ctx, const dfacto_tensor *t, int mode, int R,
                         dfacto_dtype dtype, const void *Fleaf, const void *Fmid, float *out,
                         float *carry, hipStream_t fix, hipEvent_t ev);
// Buffers of one MTTKRP when the caller provides them: returns the bytes
// of the permuted tables (0 when not relabeled), *carry_bytes the carries'.
size_t mttkrp_buffers(const dfacto_tensor *t, int mode, int R, dfacto_dtype dtype,
                      size_t *carry_bytes);
// launch_mttkrp with the caller's carries (carry_bytes) and permuted-table
// buffer (or null when not relabeled): takes no workspace of the context.
void launch_mttkrp_in(dfacto_ctx *ctx, const dfacto_tensor *t, int mode, int R,
                      dfacto_dtype dtype, const void *Fleaf, const void *Fmid, float *out,
                      float *carry, void *perm);
// residual MTTKRP over the stored entries (value x - sum_r root*mid*leaf)
void launch_mttkrp_resid(dfacto_ctx *ctx, const dfacto_tensor *t, int mode, int R,
                         dfacto_dtype dtype, const void *Fleaf, const void *Fmid,
                         const void *Froot, float *out);
// the main kernel's requests without its arithmetic (dfacto_gather_probe)
void launch_gather_probe(dfacto_ctx *ctx, const dfacto_tensor *t, int mode, int R,
                         dfacto_dtype dtype, const void *Fleaf, const void *Fmid, int pattern,
                         float *sink);
// Padded rows of relabeled gathered tables (mttkrp.hip): the row stride of
// the copies, the floats per padded output set (0 without padding), the
// bytes of `sets` such sets, and the main kernel's column count for t.
int table_stride(int R, dfacto_dtype dtype);
size_t pad_out_stride(const dfacto_tensor *t, int R, dfacto_dtype dtype);
size_t pad_out_bytes(const dfacto_tensor *t, int R, dfacto_dtype dtype, int sets);
int kernel_cols(const dfacto_tensor *t, int R, dfacto_dtype dtype);
// relabeled: the mode gathers through rank-ordered copies
MttkrpShape mttkrp_shape(int R, dfacto_dtype dtype, const void *Fleaf, const void *Fmid,
                         const float *out, bool relabeled);
bool mttkrp_small(const dfacto_tensor *t, int mode);
// chunks per work item of the grouped MTTKRP: kper per lane group
unsigned mttkrp_group_chunks_per_item(const MttkrpShape &sh, unsigned kper);
void launch_mttkrp_group(dfacto_ctx *ctx, dfacto_dtype dtype, const MttkrpShape &sh, bool small,
                         const GroupMttkrp *d_desc, const uint2 *d_items, uint32_t nitems,
                         unsigned grid, unsigned kper);
void launch_fix_group(dfacto_ctx *ctx, const MttkrpShape &sh, const GroupMttkrp *d_desc,
                      const uint4 *d_short, uint32_t nshort, const uint2 *d_empty,
                      uint32_t nempty, const uint4 *d_long, uint32_t nlong);

// dense FP64 pieces (dense.hip)
void launch_gram(dfacto_ctx *ctx, const void *F, dfacto_dtype dtype, int64_t rows, int R,
                 double *G);
void launch_solve(dfacto_ctx *ctx, int R, const double *Gp, const double *Gq, double reg,
                  double *Hinv, double *scratch, int *flag);
void launch_als_lambda(dfacto_ctx *ctx, int R, int mode, const double *Hinv, const double *MtM,
                       double *Gn, double *W, double *lambda_out, const double *GA,
                       const double *GB, double normsq, double *fit_out, double *scratch);
void launch_rowmap(dfacto_ctx *ctx, const float *M, int64_t rows, int R, const double *W,
                   void *F, dfacto_dtype dtype);
void launch_hadamard(dfacto_ctx *ctx, int R, const double *Gp, const double *Gq, double reg,
                     double *H);
void launch_gd_rows(dfacto_ctx *ctx, float *G, const void *F, dfacto_dtype dtype, int64_t rows,
                    int R, const double *H, double *inner_partial);
void launch_gd_f(dfacto_ctx *ctx, int R, const double *GA, const double *GB, const double *GC,
                 const double *inner_partial, int npartial, double normsq, double reg,
                 double *f_out);
int gd_rows_partials(int64_t rows, int R, const float *G, const void *F, dfacto_dtype dtype);
// GD step pieces: out = F - alpha G in the factor dtype; the FP64 sum of
// squares of three FP32 arrays (part: 3 * kSumsqBlocks doubles)
constexpr int kSumsqBlocks = 256;
void launch_trial_factor(dfacto_ctx *ctx, const void *F, const float *G, double alpha, void *out,
                         dfacto_dtype dtype, int64_t n);
void launch_sumsq3(dfacto_ctx *ctx, const float *const x[3], const int64_t n[3], double *part,
                   double *out);
// joint matrix completion + tensor factorization pieces (dense.hip)
constexpr int kJointSeg = 4096;  // entries per joint-ALS work item
// Row m of the joint ALS for every row of ratings mode m: S = sum v^T v +
// mu H + lam I.  Short rows use P^-1 = ws * Pinv (P = mu H + lam I; ws * I
// when Pinv is null) when *pflag == 0, the others a Cholesky of S.
void launch_joint_rows(dfacto_ctx *ctx, const dfacto_tensor *Y, int m, int64_t nrows,
                       const void *Fmid, const void *Fleaf, int R, const float *M,
                       const double *H, double mu, double lam, const double *Pinv, double ws,
                       const int *pflag, void *out, dfacto_dtype dtype, int *flag, double *part);
void launch_joint_combine(dfacto_ctx *ctx, float *G, const void *F, const float *RY, double mu,
                          double lam, int64_t n, dfacto_dtype dtype);
// fit = 1 - sqrt(max(0, ||X||^2 + lambda^T (GA*GB*GC) lambda - 2 <C diag(lambda), M>)) / ||X||
// from the stored factor C (rows x R) and its MTTKRP M; part: fit_blocks doubles
uint32_t fit_blocks(int64_t rows, int R);
void launch_fit_stored(dfacto_ctx *ctx, const void *F, dfacto_dtype dtype, const float *M,
                       int64_t rows, int R, const double *lambda, const double *GA,
                       const double *GB, const double *GC, double normsq, double *part,
                       double *fit);
// the same for every member of a group: (member, block) items, then one
// finishing block per member
void launch_fit_group(dfacto_ctx *ctx, dfacto_dtype dtype, const FitJob *d_jobs, uint32_t n,
                      const uint2 *d_items, uint32_t nitems);
void launch_dot_parts(dfacto_ctx *ctx, const void *F, const float *X, int64_t n, double *part,
                      dfacto_dtype dtype);
void launch_joint_f(dfacto_ctx *ctx, const double *ft, const double *GA, const double *GB,
                    const double *GC, int R, const double *part, int npart, double normsq_y,
                    double mu, double lam, double *f);

GramPlan gram_plan(int64_t rows, int R, const void *F, dfacto_dtype dtype);
uint32_t gram_reduce_blocks(int R);
void launch_gram_group(dfacto_ctx *ctx, dfacto_dtype dtype, int nt, bool vec,
                       const GramJob *d_jobs, const uint2 *d_vb, uint32_t nvb);
void launch_gram_reduce_group(dfacto_ctx *ctx, const GramJob *d_jobs, const uint2 *d_vb,
                              uint32_t nvb);
void launch_solve_group(dfacto_ctx *ctx, int maxR, const SolveJob *d_jobs, uint32_t n);
void launch_lambda_group(dfacto_ctx *ctx, int maxR, const LambdaJob *d_jobs, uint32_t n);
RowmapPlan rowmap_plan(int R, const float *M, const void *F, dfacto_dtype dtype, int64_t rows);
void launch_rowmap_group(dfacto_ctx *ctx, dfacto_dtype dtype, int kind, int R,
                         const RowmapJob *d_jobs, const uint2 *d_vb, uint32_t nvb);

// Make the context's device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) DF_HIP(hipSetDevice(dev));
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

template <typename F>
inline dfacto_status guarded(dfacto_ctx *ctx, F &&body) {
    if (!ctx) return DFACTO_E_INVALID;
    if (ctx->sticky) return DFACTO_E_DEVICE;
    try {
        DeviceGuard g(ctx->device);
        body();
        ctx->err.clear();
        return DFACTO_OK;
    } catch (const Error &e) {
        return fail(ctx, e.code, e.msg);
    } catch (const std::bad_alloc &) {
        return fail(ctx, DFACTO_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(ctx, DFACTO_E_DEVICE, "unexpected exception");
    }
}

inline void check_common(const dfacto_tensor *t, int R, dfacto_dtype dtype) {
    if (!t) throw Error{DFACTO_E_INVALID, "tensor is NULL"};
    if (R < 1 || R > DFACTO_MAX_R) throw Error{DFACTO_E_INVALID, "R must be in [1, 256]"};
    if (dtype != DFACTO_F32 && dtype != DFACTO_BF16) throw Error{DFACTO_E_INVALID, "bad dtype"};
}

inline size_t elem_size(dfacto_dtype d) { return d == DFACTO_BF16 ? 2 : 4; }

}  // namespace dfacto
