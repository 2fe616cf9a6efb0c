// capi.hip -- the extern "C" entry points declared in include/dfacto.h:
// argument validation, context and workspace management, and the order of
// kernel launches for MTTKRP, one CP-ALS iteration and the GD gradient.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "internal.hpp"

namespace dfacto {

dfacto_status fail(dfacto_ctx *ctx, dfacto_status code, const std::string &msg) {
    if (ctx) {
        ctx->err = msg;
        if (code == DFACTO_E_DEVICE) ctx->sticky = true;
    }
    return code;
}

void hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return;
    const dfacto_status code = (e == hipErrorOutOfMemory) ? DFACTO_E_NOMEM : DFACTO_E_DEVICE;
    (void)hipGetLastError();
    throw Error{code, std::string(what) + ": " + hipGetErrorString(e)};
}

void *ws_get(dfacto_ctx *ctx, dfacto_ctx::Slot slot, size_t bytes) {
    bytes = std::max<size_t>(bytes, 256);
    if (ctx->ws_size[slot] >= bytes) return ctx->ws[slot];
    if (ctx->frozen)
        throw Error{DFACTO_E_INVALID,
                    "a workspace would have to grow while the context is frozen"};
    const bool user = ctx->mem.has_user();
    if (ctx->ws[slot]) {
        if (user) {  // the caller's allocator orders reuse after the stream's work
            ctx->mem.free(ctx->ws[slot], ctx->stream);
        } else {
            DF_HIP(hipStreamSynchronize(ctx->stream));
            DF_HIP(hipFree(ctx->ws[slot]));
        }
        ctx->ws[slot] = nullptr;
        ctx->ws_size[slot] = 0;
    }
    const size_t grow = bytes + bytes / 8;
    void *p = nullptr;
    hip_check(user ? ctx->mem.alloc(&p, grow, ctx->stream) : hipMalloc(&p, grow),
              "workspace allocation");
    ctx->ws[slot] = p;
    ctx->ws_size[slot] = grow;
    return p;
}

void prof_mark(dfacto_ctx *ctx) {
    if (!ctx->profiling) return;
    if (ctx->ev_used == ctx->ev_pool.size()) {
        hipEvent_t e;
        DF_HIP(hipEventCreate(&e));
        ctx->ev_pool.push_back(e);
    }
    DF_HIP(hipEventRecord(ctx->ev_pool[ctx->ev_used++], ctx->stream));
}

namespace {

void check_factor(const void *p, const char *name) {
    if (!p) throw Error{DFACTO_E_INVALID, std::string(name) + " is NULL"};
}

void check_align(const void *p, dfacto_dtype d, const char *name) {
    if ((uintptr_t)p % elem_size(d) != 0)
        throw Error{DFACTO_E_INVALID, std::string(name) + " is not aligned to its element size"};
}

// the context's side stream and its fork / join events, created once
void ensure_side(dfacto_ctx *ctx) {
    if (ctx->side) return;
    DF_HIP(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
    DF_HIP(hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
    DF_HIP(hipEventCreateWithFlags(&ctx->ev_step, hipEventDisableTiming));
    DF_HIP(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
}

// launches made while alive go to `s` (the launchers use ctx->stream)
struct OnStream {
    dfacto_ctx *ctx;
    hipStream_t saved;
    OnStream(dfacto_ctx *c, hipStream_t s) : ctx(c), saved(c->stream) { c->stream = s; }
    ~OnStream() { ctx->stream = saved; }
};

int64_t max_dim(const dfacto_tensor *t) {
    return std::max(t->dims[0], std::max(t->dims[1], t->dims[2]));
}

// The workspaces that a call's launches take further down (carries of
// `carry_sets` MTTKRPs of the largest mode, the Gram partial sums of both
// streams), acquired before the call enqueues anything: a frozen context
// then fails before any work is queued.
void ws_prepare(dfacto_ctx *ctx, const dfacto_tensor *t, int R, dfacto_dtype dt, int carry_sets,
                bool grams, const dfacto_tensor *t2 = nullptr) {
    int64_t cmax = 1;
    for (int m = 0; m < 3; ++m) {
        cmax = std::max<int64_t>(cmax, t->mode[m].nchunk);
        if (t2) cmax = std::max<int64_t>(cmax, t2->mode[m].nchunk);
    }
    const int kc = std::max(kernel_cols(t, R, dt), t2 ? kernel_cols(t2, R, dt) : R);
    ws_get(ctx, dfacto_ctx::kCarry, sizeof(float) * (size_t)carry_sets * cmax * kc);
    const size_t pb = perm_bytes(t, R, dt);
    if (pb) ws_get(ctx, dfacto_ctx::kPerm, pb);
    if (pad_out_stride(t, R, dt)) ws_get(ctx, dfacto_ctx::kPadOut, pad_out_bytes(t, R, dt, carry_sets));
    if (grams) {
        ws_get(ctx, dfacto_ctx::kPartial, sizeof(double) * 256 * (size_t)R * R);
        ws_get(ctx, dfacto_ctx::kPartialSide, sizeof(double) * 256 * (size_t)R * R);
    }
}

// small FP64 workspace layout (units of doubles)
struct Small {
    double *G[3], *Hinv, *W, *MtM, *solve_scratch, *lam_scratch, *H[3], *part0, *part_dummy;
    double *GT[3], *HT, *part_t, *scal;  // GD step: trial Grams, trial H, partials, scalars
    int *flag;
};

Small small_ws(dfacto_ctx *ctx, int R) {
    const size_t RR = (size_t)R * R;
    const size_t n = 3 * RR + 3 * RR + 3 * RR + (4 * RR + R) + 3 * RR + 2 * 8192 + 4 * RR +
                     8192 + 3 * kSumsqBlocks + 8 + 64;
    double *b = (double *)ws_get(ctx, dfacto_ctx::kSmall, sizeof(double) * n);
    Small s;
    size_t o = 0;
    for (int m = 0; m < 3; ++m) s.G[m] = b + o, o += RR;
    s.Hinv = b + o, o += RR;
    s.W = b + o, o += RR;
    s.MtM = b + o, o += RR;
    s.solve_scratch = b + o, o += 3 * RR;
    s.lam_scratch = b + o, o += 4 * RR + R;
    for (int m = 0; m < 3; ++m) s.H[m] = b + o, o += RR;
    s.part0 = b + o, o += 8192;
    s.part_dummy = b + o, o += 8192;
    for (int m = 0; m < 3; ++m) s.GT[m] = b + o, o += RR;
    s.HT = b + o, o += RR;
    s.part_t = b + o, o += 8192;
    s.scal = b + o, o += 3 * kSumsqBlocks + 8;  // partials, then gnorm2, f0, f_trial
    s.flag = (int *)(b + o);
    return s;
}

}  // namespace
}  // namespace dfacto

namespace dfacto {

dfacto_status build_flattenings_impl(dfacto_ctx *ctx, const int64_t dims[3], int64_t nnz,
                                     const uint32_t *d_i, const uint32_t *d_j,
                                     const uint32_t *d_k, const float *d_val, dfacto_tensor **out,
                                     bool async_alloc, int flags, int chunk_len) {
    if (out) *out = nullptr;
    return guarded(ctx, [&] {
        if (!out || !dims) throw Error{DFACTO_E_INVALID, "dims or out is NULL"};
        for (int m = 0; m < 3; ++m)
            if (dims[m] < 1 || dims[m] > DFACTO_MAX_DIM)
                throw Error{DFACTO_E_INVALID, "every dimension must be in [1, 2^30]"};
        if (nnz < 0) throw Error{DFACTO_E_INVALID, "nnz is negative"};
        if (nnz > 0 && (!d_i || !d_j || !d_k || !d_val))
            throw Error{DFACTO_E_INVALID, "coordinate or value array is NULL"};
        if (nnz >= (int64_t)0xFFFFFFFFu - (1 << 20))
            throw Error{DFACTO_E_UNSUPPORTED, "nnz must be below 2^32 - 2^20"};
        if (flags & ~(DFACTO_BUILD_RELABEL | DFACTO_BUILD_NO_RELABEL) ||
            (flags & DFACTO_BUILD_RELABEL && flags & DFACTO_BUILD_NO_RELABEL))
            throw Error{DFACTO_E_INVALID, "bad build flags"};
        if (chunk_len != 0 && (chunk_len < 2 * kFiberCap || chunk_len > (1 << 20)))
            throw Error{DFACTO_E_INVALID, "chunk_len must be 0 or in [256, 2^20]"};
        dfacto_tensor *t = new dfacto_tensor();
        t->chunk_len = chunk_len ? chunk_len : DFACTO_CHUNK_DEFAULT;
        t->relabel = (flags & DFACTO_BUILD_RELABEL) ||
                     (!(flags & DFACTO_BUILD_NO_RELABEL) && nnz >= kRelabelMinNnz &&
                      nnz >= kRelabelPerRow * (dims[0] + dims[1] + dims[2]));
        t->device = ctx->device;
        if (async_alloc || ctx->mem.has_user()) {
            t->alloc_stream = ctx->stream;
            t->mem = ctx->mem;
        }
        for (int m = 0; m < 3; ++m) t->dims[m] = dims[m];
        t->nnz = nnz;
        // Without a memory source of the caller's, the build's temporaries
        // come from a pool of the context that keeps freed memory mapped
        // until the build ends (memory given back to the device is mapped
        // afresh, and cleared, at each later allocation), then gives it all
        // back.
        hipMemPool_t pool = nullptr;
        if (!ctx->mem.has_user() && !ctx->mem.pool) {
            if (!ctx->build_pool) {
                hipMemPoolProps props{};
                props.allocType = hipMemAllocationTypePinned;
                props.location.type = hipMemLocationTypeDevice;
                props.location.id = ctx->device;
                uint64_t keep = UINT64_MAX;
                if (hipMemPoolCreate(&ctx->build_pool, &props) != hipSuccess ||
                    hipMemPoolSetAttribute(ctx->build_pool, hipMemPoolAttrReleaseThreshold,
                                           &keep) != hipSuccess) {
                    (void)hipGetLastError();  // fall back to the default pool
                    if (ctx->build_pool) (void)hipMemPoolDestroy(ctx->build_pool);
                    ctx->build_pool = nullptr;
                }
            }
            pool = ctx->build_pool;
        }
        auto drop_pool = [&] {
            if (!pool) return;
            ctx->mem.pool = nullptr;
            (void)hipStreamSynchronize(ctx->stream);  // the temporaries' frees
            (void)hipMemPoolTrimTo(pool, 0);
        };
        ctx->mem.pool = pool ? pool : ctx->mem.pool;
        try {
            // the build's small temporaries come from an arena whose chunks
            // go back (stream-ordered) before the pool is emptied
            Arena arena(ctx->stream, ctx->mem);
            ctx->mem.arena = &arena;
            try {
                build_tensor(ctx, t, d_i, d_j, d_k, d_val);
            } catch (...) {
                ctx->mem.arena = nullptr;
                throw;
            }
            ctx->mem.arena = nullptr;
        } catch (...) {
            // copies into the tensor's host fields may still be pending
            (void)hipStreamSynchronize(ctx->stream);
            drop_pool();
            dfacto_tensor_destroy(t);
            throw;
        }
        drop_pool();
        *out = t;
    });
}

dfacto_status build_flattenings_async_alloc(dfacto_ctx *ctx, const int64_t dims[3], int64_t nnz,
                                            const uint32_t *d_i, const uint32_t *d_j,
                                            const uint32_t *d_k, const float *d_val,
                                            dfacto_tensor **out) {
    return build_flattenings_impl(ctx, dims, nnz, d_i, d_j, d_k, d_val, out, true,
                                  DFACTO_BUILD_NO_RELABEL, 0);
}

}  // namespace dfacto

using namespace dfacto;

extern "C" {

dfacto_status dfacto_ctx_create(int device, void *hip_stream, const dfacto_allocator *alloc,
                                dfacto_ctx **out) {
    if (!out) return DFACTO_E_INVALID;
    *out = nullptr;
    if (alloc && (!alloc->alloc || !alloc->free)) return DFACTO_E_INVALID;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return DFACTO_E_DEVICE;
    }
    if (device < 0 || device >= n) return DFACTO_E_INVALID;
    dfacto_ctx *ctx = new (std::nothrow) dfacto_ctx();
    if (!ctx) return DFACTO_E_NOMEM;
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    if (alloc) ctx->mem.user = *alloc;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->num_cu = prop.multiProcessorCount;
    *out = ctx;
    return DFACTO_OK;
}

dfacto_status dfacto_ctx_set_stream(dfacto_ctx *ctx, void *hip_stream) {
    if (!ctx) return DFACTO_E_INVALID;
    ctx->stream = (hipStream_t)hip_stream;
    return DFACTO_OK;
}

dfacto_status dfacto_ctx_synchronize(dfacto_ctx *ctx) {
    return guarded(ctx, [&] { DF_HIP(hipStreamSynchronize(ctx->stream)); });
}

dfacto_status dfacto_ctx_freeze(dfacto_ctx *ctx, int on) {
    if (!ctx) return DFACTO_E_INVALID;
    ctx->frozen = on != 0;
    return DFACTO_OK;
}

void dfacto_ctx_destroy(dfacto_ctx *ctx) {
    if (!ctx) return;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->side) {
        (void)hipStreamSynchronize(ctx->side);
        (void)hipStreamDestroy(ctx->side);
    }
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    if (ctx->ev_step) (void)hipEventDestroy(ctx->ev_step);
    for (int s = 0; s < dfacto_ctx::kNumSlots; ++s) {
        if (!ctx->ws[s]) continue;
        if (ctx->mem.has_user()) ctx->mem.free(ctx->ws[s], ctx->stream);
        else (void)hipFree(ctx->ws[s]);
    }
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    if (ctx->build_pool) (void)hipMemPoolDestroy(ctx->build_pool);
    if (prev >= 0) (void)hipSetDevice(prev);
    delete ctx;
}

const char *dfacto_last_error(const dfacto_ctx *ctx) {
    if (!ctx) return "context is NULL";
    return ctx->err.c_str();
}

dfacto_status dfacto_build_flattenings(dfacto_ctx *ctx, const int64_t dims[3], int64_t nnz,
                                       const uint32_t *d_i, const uint32_t *d_j,
                                       const uint32_t *d_k, const float *d_val,
                                       dfacto_tensor **out) {
    return build_flattenings_impl(ctx, dims, nnz, d_i, d_j, d_k, d_val, out, false, 0, 0);
}

dfacto_status dfacto_build_flattenings_ex(dfacto_ctx *ctx, const int64_t dims[3], int64_t nnz,
                                          const uint32_t *d_i, const uint32_t *d_j,
                                          const uint32_t *d_k, const float *d_val, int flags,
                                          int chunk_len, dfacto_tensor **out) {
    return build_flattenings_impl(ctx, dims, nnz, d_i, d_j, d_k, d_val, out, false, flags,
                                  chunk_len);
}

dfacto_status dfacto_tensor_get_info(const dfacto_tensor *t, dfacto_tensor_info *info) {
    if (!t || !info) return DFACTO_E_INVALID;
    memset(info, 0, sizeof(*info));
    for (int m = 0; m < 3; ++m) {
        info->dims[m] = t->dims[m];
        info->nfib[m] = t->mode[m].nfib;
        info->nroot[m] = t->mode[m].nroot;
        info->nentry[m] = t->mode[m].nentry;
        info->nchunk[m] = t->mode[m].nchunk;
    }
    info->relabeled = t->relabel ? 1 : 0;
    info->chunk_len = t->chunk_len;
    info->nnz = t->nnz;
    info->normsq = t->normsq;
    info->bytes = t->bytes;
    return DFACTO_OK;
}

dfacto_status dfacto_tensor_export(dfacto_ctx *ctx, const dfacto_tensor *t, int mode,
                                   uint32_t *h_root_id, int64_t *h_root_ptr, uint32_t *h_fib_mid,
                                   int64_t *h_fib_ptr, uint32_t *h_leaf, float *h_val) {
    return guarded(ctx, [&] {
        if (!t) throw Error{DFACTO_E_INVALID, "tensor is NULL"};
        if (mode < 0 || mode > 2) throw Error{DFACTO_E_INVALID, "mode must be 0, 1 or 2"};
        if (!h_root_id || !h_root_ptr || !h_fib_mid || !h_fib_ptr || !h_leaf || !h_val)
            throw Error{DFACTO_E_INVALID, "an output array is NULL"};
        const ModeData &md = t->mode[mode];
        std::vector<uint2> st((size_t)md.nentry);
        if (md.nentry > 0) {
            DF_HIP(hipMemcpyAsync(st.data(), md.stream, sizeof(uint2) * md.nentry,
                                  hipMemcpyDeviceToHost, ctx->stream));
        }
        // relabeled gathers: back to the factor rows
        std::vector<uint32_t> pl, pm;
        if (md.perm_leaf) {
            pl.resize((size_t)t->dims[md.leaf]);
            pm.resize((size_t)t->dims[md.mid]);
            DF_HIP(hipMemcpyAsync(pl.data(), md.perm_leaf, sizeof(uint32_t) * pl.size(),
                                  hipMemcpyDeviceToHost, ctx->stream));
            DF_HIP(hipMemcpyAsync(pm.data(), md.perm_mid, sizeof(uint32_t) * pm.size(),
                                  hipMemcpyDeviceToHost, ctx->stream));
        }
        DF_HIP(hipStreamSynchronize(ctx->stream));
        if (md.perm_leaf)
            for (uint2 &w : st) {
                if (w.x & kHdrBit) w.x = (w.x & ~kIdxMask) | pm[w.x & kIdxMask];
                else w.x = pl[w.x];
            }
        int64_t nr = 0, nf = 0, ne = 0;
        uint32_t last_mid = 0;
        for (const uint2 &w : st) {
            if (w.x & kHdrBit) {
                const uint32_t mid = w.x & kIdxMask;
                const bool root = (w.x & kRootBit) != 0;
                if (root) {
                    h_root_id[nr] = w.y;
                    h_root_ptr[nr] = nf;
                    ++nr;
                }
                if (root || mid != last_mid) {  // else: continuation segment of the same fiber
                    h_fib_mid[nf] = mid;
                    h_fib_ptr[nf] = ne;
                    ++nf;
                }
                last_mid = mid;
            } else {
                h_leaf[ne] = w.x;
                uint32_t b = w.y;
                memcpy(&h_val[ne], &b, sizeof(float));
                ++ne;
            }
        }
        h_root_ptr[nr] = nf;
        h_fib_ptr[nf] = ne;
        if (nr != md.nroot || nf != md.nfib || ne != t->nnz)
            throw Error{DFACTO_E_DEVICE, "flattening stream is inconsistent with its counts"};
    });
}

dfacto_status dfacto_tensor_gather_order(dfacto_ctx *ctx, const dfacto_tensor *t, int mode,
                                         int table, uint32_t *h_order) {
    return guarded(ctx, [&] {
        if (!t || !h_order) throw Error{DFACTO_E_INVALID, "tensor or output is NULL"};
        if (mode < 0 || mode > 2) throw Error{DFACTO_E_INVALID, "mode must be 0, 1 or 2"};
        if (table != 0 && table != 1) throw Error{DFACTO_E_INVALID, "table must be 0 or 1"};
        const ModeData &md = t->mode[mode];
        if (!md.perm_leaf) throw Error{DFACTO_E_INVALID, "the tensor is not relabeled"};
        const uint32_t *src = table == 0 ? md.perm_leaf : md.perm_mid;
        const int64_t rows = t->dims[table == 0 ? md.leaf : md.mid];
        DF_HIP(hipMemcpyAsync(h_order, src, sizeof(uint32_t) * (size_t)rows,
                              hipMemcpyDeviceToHost, ctx->stream));
        DF_HIP(hipStreamSynchronize(ctx->stream));
    });
}

void dfacto_tensor_destroy(dfacto_tensor *t) {
    if (!t) return;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(t->device);
    if (t->alloc_stream) {  // stream-ordered memory: free after the stream's work
        for (void *p : t->allocations) t->mem.free(p, t->alloc_stream);
    } else {
        (void)hipDeviceSynchronize();
        for (void *p : t->allocations) (void)hipFree(p);
    }
    if (prev >= 0) (void)hipSetDevice(prev);
    delete t;
}

dfacto_status dfacto_mttkrp(dfacto_ctx *ctx, const dfacto_tensor *t, int mode, int R,
                            dfacto_dtype dtype, const void *const d_F[3], float *d_out) {
    return guarded(ctx, [&] {
        check_common(t, R, dtype);
        if (mode < 0 || mode > 2) throw Error{DFACTO_E_INVALID, "mode must be 0, 1 or 2"};
        if (!d_F || !d_out) throw Error{DFACTO_E_INVALID, "factor array or output is NULL"};
        const ModeData &md = t->mode[mode];
        check_factor(d_F[md.leaf], "leaf factor");
        check_factor(d_F[md.mid], "mid factor");
        check_align(d_F[md.leaf], dtype, "leaf factor");
        check_align(d_F[md.mid], dtype, "mid factor");
        if ((uintptr_t)d_out % 4) throw Error{DFACTO_E_INVALID, "output is not 4-byte aligned"};
        ws_prepare(ctx, t, R, dtype, 1, false);
        launch_mttkrp(ctx, t, mode, R, dtype, d_F[md.leaf], d_F[md.mid], d_out);
    });
}

dfacto_status dfacto_gather_probe(dfacto_ctx *ctx, const dfacto_tensor *t, int mode, int R,
                                  dfacto_dtype dtype, const void *const d_F[3], int pattern,
                                  float *d_sink) {
    return guarded(ctx, [&] {
        check_common(t, R, dtype);
        if (mode < 0 || mode > 2) throw Error{DFACTO_E_INVALID, "mode must be 0, 1 or 2"};
        if (pattern < 0 || pattern > 9) throw Error{DFACTO_E_INVALID, "pattern must be 0 .. 9"};
        if (!d_F || !d_sink) throw Error{DFACTO_E_INVALID, "factor array or sink is NULL"};
        const ModeData &md = t->mode[mode];
        check_factor(d_F[md.leaf], "leaf factor");
        check_factor(d_F[md.mid], "mid factor");
        check_align(d_F[md.leaf], dtype, "leaf factor");
        check_align(d_F[md.mid], dtype, "mid factor");
        if ((uintptr_t)d_sink % 16) throw Error{DFACTO_E_INVALID, "sink is not 16-byte aligned"};
        launch_gather_probe(ctx, t, mode, R, dtype, d_F[md.leaf], d_F[md.mid], pattern, d_sink);
    });
}

dfacto_status dfacto_als_iter(dfacto_ctx *ctx, const dfacto_tensor *t, int R, dfacto_dtype dtype,
                              double reg, void *const d_F[3], double *d_lambda, double *d_fit) {
    return guarded(ctx, [&] {
        check_common(t, R, dtype);
        if (!d_F || !d_lambda || !d_fit) throw Error{DFACTO_E_INVALID, "NULL argument"};
        if (!(reg >= 0.0)) throw Error{DFACTO_E_INVALID, "reg must be >= 0"};
        for (int m = 0; m < 3; ++m) {
            check_factor(d_F[m], "factor");
            check_align(d_F[m], dtype, "factor");
        }
        Small sw = small_ws(ctx, R);
        float *M = (float *)ws_get(ctx, dfacto_ctx::kM, sizeof(float) * (size_t)max_dim(t) * R);
        ws_prepare(ctx, t, R, dtype, 1, true);
        ensure_side(ctx);
        // Mode n's R x R solve needs only the other modes' Grams, final once
        // mode n - 1's factor and Gram are: it runs on the side stream beside
        // mode n's MTTKRP and is joined before mode n's lambda step.  Mode 0's
        // solve follows the Grams of F[1] and F[2], also formed there.  The
        // MTTKRP is enqueued before the side stream's part.
        for (int n = 0; n < 3; ++n) {
            const ModeData &md = t->mode[n];
            DF_HIP(hipEventRecord(ctx->ev_fork, ctx->stream));
            launch_mttkrp(ctx, t, n, R, dtype, d_F[md.leaf], d_F[md.mid], M);
            DF_HIP(hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0));
            {
                OnStream on(ctx, ctx->side);
                if (n == 0) {
                    launch_gram(ctx, d_F[1], dtype, t->dims[1], R, sw.G[1]);
                    launch_gram(ctx, d_F[2], dtype, t->dims[2], R, sw.G[2]);
                } else if (dtype == DFACTO_BF16) {
                    // the Gram of the previous mode's stored (rounded) factor
                    launch_gram(ctx, d_F[n - 1], dtype, t->dims[n - 1], R, sw.G[n - 1]);
                }
                launch_solve(ctx, R, sw.G[(n + 1) % 3], sw.G[(n + 2) % 3], reg, sw.Hinv,
                             sw.solve_scratch, sw.flag + n);
            }
            DF_HIP(hipEventRecord(ctx->ev_join, ctx->side));
            launch_gram(ctx, M, DFACTO_F32, t->dims[n], R, sw.MtM);
            DF_HIP(hipStreamWaitEvent(ctx->stream, ctx->ev_join, 0));
            // writes G[n] (the new factor's Gram) and W; reads H^-1
            launch_als_lambda(ctx, R, n, sw.Hinv, sw.MtM, sw.G[n], sw.W, d_lambda, sw.G[0],
                              sw.G[1], t->normsq, d_fit, sw.lam_scratch);
            launch_rowmap(ctx, M, t->dims[n], R, sw.W, d_F[n], dtype);
            // A BF16-stored factor differs from the FP64 one by its rounding;
            // the next modes' normal equations must use the Gram of what the
            // next MTTKRPs read, so it is formed from the stored factor (for
            // modes 0 and 1 on the side stream beside the next MTTKRP, ahead
            // of the next solve); and the fit is that of the stored factors
            // (lambda from the FP64 ones).
            if (dtype == DFACTO_BF16 && n == 2) {
                launch_gram(ctx, d_F[2], dtype, t->dims[2], R, sw.G[2]);
                launch_fit_stored(ctx, d_F[2], dtype, M, t->dims[2], R, d_lambda, sw.G[0],
                                  sw.G[1], sw.G[2], t->normsq, sw.part0, d_fit);
            }
        }
    });
}

dfacto_status dfacto_gd_grad(dfacto_ctx *ctx, const dfacto_tensor *t, int R, dfacto_dtype dtype,
                             double reg, const void *const d_F[3], float *const d_G[3],
                             double *d_f) {
    return guarded(ctx, [&] {
        check_common(t, R, dtype);
        if (!d_F || !d_G || !d_f) throw Error{DFACTO_E_INVALID, "NULL argument"};
        if (!(reg >= 0.0)) throw Error{DFACTO_E_INVALID, "reg must be >= 0"};
        for (int m = 0; m < 3; ++m) {
            check_factor(d_F[m], "factor");
            check_align(d_F[m], dtype, "factor");
            if (!d_G[m]) throw Error{DFACTO_E_INVALID, "gradient output is NULL"};
            if ((uintptr_t)d_G[m] % 4) throw Error{DFACTO_E_INVALID, "gradient not aligned"};
        }
        Small sw = small_ws(ctx, R);
        ws_prepare(ctx, t, R, dtype, 3, true);
        ensure_side(ctx);
        // the three MTTKRPs' main kernels run back to back on the main
        // stream, each with carries of its own; the Grams, each mode's carry
        // fix-ups and its gradient rows (which need only that mode's
        // MTTKRP) run on the side stream beside the next MTTKRP; joined at
        // the end
        const hipStream_t main = ctx->stream;
        int64_t cmax = 1;
        for (int m = 0; m < 3; ++m) cmax = std::max<int64_t>(cmax, t->mode[m].nchunk);
        const size_t cstride = (size_t)cmax * kernel_cols(t, R, dtype);
        float *carry =
            (float *)ws_get(ctx, dfacto_ctx::kCarry, sizeof(float) * 3 * cstride);
        DF_HIP(hipEventRecord(ctx->ev_fork, main));
        DF_HIP(hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0));
        {
            OnStream on(ctx, ctx->side);
            for (int m = 0; m < 3; ++m) launch_gram(ctx, d_F[m], dtype, t->dims[m], R, sw.G[m]);
            for (int n = 0; n < 3; ++n)
                launch_hadamard(ctx, R, sw.G[(n + 1) % 3], sw.G[(n + 2) % 3], reg, sw.H[n]);
        }
        for (int n = 0; n < 3; ++n) {
            const ModeData &md = t->mode[n];
            launch_mttkrp_split(ctx, t, n, R, dtype, d_F[md.leaf], d_F[md.mid], d_G[n],
                                carry + n * cstride, ctx->side, ctx->ev_step);
            OnStream on(ctx, ctx->side);
            launch_gd_rows(ctx, d_G[n], d_F[n], dtype, t->dims[n], R, sw.H[n],
                           n == 0 ? sw.part0 : sw.part_dummy);
        }
        {
            OnStream on(ctx, ctx->side);
            launch_gd_f(ctx, R, sw.G[0], sw.G[1], sw.G[2], sw.part0,
                        gd_rows_partials(t->dims[0], R, d_G[0], d_F[0], dtype),
                        t->normsq, reg, d_f);
        }
        DF_HIP(hipEventRecord(ctx->ev_join, ctx->side));
        DF_HIP(hipStreamWaitEvent(main, ctx->ev_join, 0));
    });
}

dfacto_status dfacto_gd_step(dfacto_ctx *ctx, const dfacto_tensor *t, int R, dfacto_dtype dtype,
                             double reg, void *const d_F[3], float *const d_G[3],
                             const dfacto_linesearch *ls, dfacto_gd_step_info *info) {
    return guarded(ctx, [&] {
        if (!ls || !info) throw Error{DFACTO_E_INVALID, "NULL argument"};
        if (!(ls->alpha0 > 0.0) || !std::isfinite(ls->alpha0))
            throw Error{DFACTO_E_INVALID, "alpha0 must be positive and finite"};
        if (!(ls->shrink > 0.0 && ls->shrink < 1.0))
            throw Error{DFACTO_E_INVALID, "shrink must be in (0, 1)"};
        if (!(ls->c > 0.0 && ls->c < 1.0)) throw Error{DFACTO_E_INVALID, "c must be in (0, 1)"};
        if (ls->max_trials < 1 || ls->max_trials > 1000)
            throw Error{DFACTO_E_INVALID, "max_trials must be in [1, 1000]"};
        check_common(t, R, dtype);
        *info = dfacto_gd_step_info{};
        // the gradient and f at the input point (validates the other arguments);
        // the gradient call uses the same small workspace (same R: same buffer)
        Small sw = small_ws(ctx, R);
        double *d_gn2 = sw.scal + 3 * kSumsqBlocks, *d_f0 = d_gn2 + 1, *d_ft = d_gn2 + 2;
        {
            const dfacto_status st = dfacto_gd_grad(ctx, t, R, dtype, reg, d_F, d_G, d_f0);
            if (st != DFACTO_OK) throw Error{st, ctx->err};
        }
        const int64_t n[3] = {t->dims[0] * R, t->dims[1] * R, t->dims[2] * R};
        const float *g[3] = {d_G[0], d_G[1], d_G[2]};
        launch_sumsq3(ctx, g, n, sw.scal, d_gn2);
        // trial factors and the mode-0 MTTKRP of the trial point
        const size_t es = elem_size(dtype);
        size_t off[4], o = 0;
        for (int m = 0; m < 3; ++m) off[m] = o, o += ((size_t)n[m] * es + 255) & ~(size_t)255;
        off[3] = o, o += (size_t)n[0] * 4;
        char *wt = (char *)ws_get(ctx, dfacto_ctx::kTrial, o);
        void *T[3] = {wt + off[0], wt + off[1], wt + off[2]};
        float *M = (float *)(wt + off[3]);
        double host[2];
        DF_HIP(hipMemcpyAsync(host, d_gn2, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        DF_HIP(hipStreamSynchronize(ctx->stream));
        const double gn2 = host[0], f0 = host[1];
        info->f0 = f0;
        info->f = f0;
        info->gnorm2 = gn2;
        const ModeData &md = t->mode[0];
        double alpha = ls->alpha0;
        for (int trial = 0; trial < ls->max_trials; ++trial) {
            for (int m = 0; m < 3; ++m) launch_trial_factor(ctx, d_F[m], d_G[m], alpha, T[m], dtype, n[m]);
            // f at the trial point, as in dfacto_gd_grad: Grams, the mode-0
            // MTTKRP, <T_0, M> by the gradient-row pass, then the combination
            for (int m = 0; m < 3; ++m) launch_gram(ctx, T[m], dtype, t->dims[m], R, sw.GT[m]);
            launch_hadamard(ctx, R, sw.GT[1], sw.GT[2], reg, sw.HT);
            launch_mttkrp(ctx, t, 0, R, dtype, T[md.leaf], T[md.mid], M);
            launch_gd_rows(ctx, M, T[0], dtype, t->dims[0], R, sw.HT, sw.part_t);
            launch_gd_f(ctx, R, sw.GT[0], sw.GT[1], sw.GT[2], sw.part_t,
                        gd_rows_partials(t->dims[0], R, M, T[0], dtype), t->normsq, reg, d_ft);
            double ft = 0.0;
            DF_HIP(hipMemcpyAsync(&ft, d_ft, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
            DF_HIP(hipStreamSynchronize(ctx->stream));
            info->trials = trial + 1;
            if (ft <= f0 - ls->c * alpha * gn2) {  // Armijo: sufficient decrease
                for (int m = 0; m < 3; ++m)
                    DF_HIP(hipMemcpyAsync(d_F[m], T[m], (size_t)n[m] * es,
                                          hipMemcpyDeviceToDevice, ctx->stream));
                info->f = ft;
                info->alpha = alpha;
                info->accepted = 1;
                break;
            }
            alpha *= ls->shrink;
        }
    });
}

// ---- joint matrix completion + tensor factorization -----------------------

dfacto_status dfacto_build_ratings(dfacto_ctx *ctx, const int64_t dims[2], int64_t n,
                                   const uint32_t *d_i, const uint32_t *d_j, const float *d_y,
                                   dfacto_tensor **out) {
    if (out) *out = nullptr;
    return guarded(ctx, [&] {
        if (!out || !dims) throw Error{DFACTO_E_INVALID, "dims or out is NULL"};
        if (n < 0) throw Error{DFACTO_E_INVALID, "n is negative"};
        uint32_t *k0 = nullptr;
        hip_check(ctx->mem.alloc((void **)&k0, sizeof(uint32_t) * (size_t)std::max<int64_t>(n, 1),
                                 ctx->stream),
                  "ratings staging");
        DF_HIP(hipMemsetAsync(k0, 0, sizeof(uint32_t) * (size_t)std::max<int64_t>(n, 1),
                              ctx->stream));
        const int64_t d3[3] = {dims[0], dims[1], 1};
        dfacto_tensor *t = nullptr;
        // the joint rows read the ratings' streams directly: plain indices
        const dfacto_status st = dfacto_build_flattenings_ex(ctx, d3, n, d_i, d_j, k0, d_y,
                                                             DFACTO_BUILD_NO_RELABEL, 0, &t);
        ctx->mem.free(k0, ctx->stream);
        if (st != DFACTO_OK) throw Error{st, ctx->err};
        try {
            build_row_ranges(ctx, t);
        } catch (...) {
            dfacto_tensor_destroy(t);
            throw;
        }
        t->ratings = true;
        *out = t;
    });
}

namespace {

void check_joint(const dfacto_tensor *X, const dfacto_tensor *Y, int R, dfacto_dtype dtype,
                 double mu, double lam) {
    check_common(X, R, dtype);
    if (!Y) throw Error{DFACTO_E_INVALID, "ratings matrix is NULL"};
    if (!Y->ratings) throw Error{DFACTO_E_INVALID, "Y was not built by dfacto_build_ratings"};
    if (Y->dims[0] != X->dims[0] || Y->dims[1] != X->dims[1])
        throw Error{DFACTO_E_INVALID, "Y must be users x items of X (dims[0] x dims[1])"};
    if (Y->device != X->device) throw Error{DFACTO_E_INVALID, "X and Y on different devices"};
    if (!(mu >= 0.0) || !(lam >= 0.0)) throw Error{DFACTO_E_INVALID, "mu and lam must be >= 0"};
}

// a 1 x R row of ones in the factor dtype: the third "factor" of the
// ratings matrix seen as a users x items x 1 tensor
void *ones_row(dfacto_ctx *ctx, int R, dfacto_dtype dtype, void *dst) {
#define DF_X8(v) v, v, v, v, v, v, v, v
#define DF_X64(v) DF_X8(v), DF_X8(v), DF_X8(v), DF_X8(v), DF_X8(v), DF_X8(v), DF_X8(v), DF_X8(v)
    static_assert(DFACTO_MAX_R == 256, "ones table size");
    static const float f1[256] = {DF_X64(1.f), DF_X64(1.f), DF_X64(1.f), DF_X64(1.f)};
    static const uint16_t b1[256] = {DF_X64(0x3F80u), DF_X64(0x3F80u), DF_X64(0x3F80u),
                                     DF_X64(0x3F80u)};  // BF16 1.0
#undef DF_X64
#undef DF_X8
    DF_HIP(hipMemcpyAsync(dst, dtype == DFACTO_F32 ? (const void *)f1 : (const void *)b1,
                          (size_t)R * elem_size(dtype), hipMemcpyHostToDevice, ctx->stream));
    return dst;
}

}  // namespace

dfacto_status dfacto_joint_grad(dfacto_ctx *ctx, const dfacto_tensor *X, const dfacto_tensor *Y,
                                int R, dfacto_dtype dtype, double mu, double lam,
                                const void *const d_F[3], float *const d_G[3], double *d_f) {
    return guarded(ctx, [&] {
        check_joint(X, Y, R, dtype, mu, lam);
        if (!d_F || !d_G || !d_f) throw Error{DFACTO_E_INVALID, "NULL argument"};
        for (int m = 0; m < 3; ++m) {
            check_factor(d_F[m], "factor");
            check_align(d_F[m], dtype, "factor");
            if (!d_G[m]) throw Error{DFACTO_E_INVALID, "gradient output is NULL"};
            if ((uintptr_t)d_G[m] % 4) throw Error{DFACTO_E_INVALID, "gradient not aligned"};
        }
        Small sw = small_ws(ctx, R);
        // workspace: ones row, the ratings' residual MTTKRPs of modes 0 and
        // 1, the plain one of mode 0, partial sums, the tensor objective
        const size_t d0 = (size_t)X->dims[0] * R, d1 = (size_t)X->dims[1] * R;
        auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
        const size_t o_ry0 = al(4 * (size_t)R), o_ry1 = o_ry0 + al(4 * d0);
        const size_t o_my0 = o_ry1 + al(4 * d1);
        const size_t o_part = o_my0 + al(4 * d0), o_ft = o_part + al(8 * 2 * kSumsqBlocks);
        char *w = (char *)ws_get(ctx, dfacto_ctx::kJoint, o_ft + 256);
        ws_prepare(ctx, X, R, dtype, 1, true, Y);
        void *one = ones_row(ctx, R, dtype, w);
        float *RY0 = (float *)(w + o_ry0), *RY1 = (float *)(w + o_ry1), *MY0 = (float *)(w + o_my0);
        double *part = (double *)(w + o_part), *ft = (double *)(w + o_ft);
        // tensor part, as dfacto_gd_grad with reg = 0: G_n = -M_n + F_n H_n
        for (int m = 0; m < 3; ++m) launch_gram(ctx, d_F[m], dtype, X->dims[m], R, sw.G[m]);
        for (int n = 0; n < 3; ++n)
            launch_hadamard(ctx, R, sw.G[(n + 1) % 3], sw.G[(n + 2) % 3], 0.0, sw.H[n]);
        for (int n = 0; n < 3; ++n) {
            const ModeData &md = X->mode[n];
            launch_mttkrp(ctx, X, n, R, dtype, d_F[md.leaf], d_F[md.mid], d_G[n]);
            launch_gd_rows(ctx, d_G[n], d_F[n], dtype, X->dims[n], R, sw.H[n],
                           n == 0 ? sw.part0 : sw.part_dummy);
        }
        launch_gd_f(ctx, R, sw.G[0], sw.G[1], sw.G[2], sw.part0,
                    gd_rows_partials(X->dims[0], R, d_G[0], d_F[0], dtype), X->normsq, 0.0, ft);
        // ratings part: Y's mode 0 is (user, 1, item), mode 1 (item, user, 1)
        launch_mttkrp_resid(ctx, Y, 0, R, dtype, d_F[1], one, d_F[0], RY0);
        launch_mttkrp_resid(ctx, Y, 1, R, dtype, one, d_F[0], d_F[1], RY1);
        launch_mttkrp(ctx, Y, 0, R, dtype, d_F[1], one, MY0);
        launch_joint_combine(ctx, d_G[0], d_F[0], RY0, mu, lam, (int64_t)d0, dtype);
        launch_joint_combine(ctx, d_G[1], d_F[1], RY1, mu, lam, (int64_t)d1, dtype);
        launch_joint_combine(ctx, d_G[2], d_F[2], nullptr, mu, lam, X->dims[2] * R, dtype);
        launch_dot_parts(ctx, d_F[0], MY0, (int64_t)d0, part, dtype);
        launch_dot_parts(ctx, d_F[0], RY0, (int64_t)d0, part + kSumsqBlocks, dtype);
        launch_joint_f(ctx, ft, sw.G[0], sw.G[1], sw.G[2], R, part, 2 * kSumsqBlocks, Y->normsq,
                       mu, lam, d_f);
    });
}

dfacto_status dfacto_joint_als_iter(dfacto_ctx *ctx, const dfacto_tensor *X,
                                    const dfacto_tensor *Y, int R, dfacto_dtype dtype, double mu,
                                    double lam, void *const d_F[3]) {
    return guarded(ctx, [&] {
        check_joint(X, Y, R, dtype, mu, lam);
        if (R > 32) throw Error{DFACTO_E_UNSUPPORTED, "joint ALS supports R <= 32"};
        if (!(lam > 0.0)) throw Error{DFACTO_E_INVALID, "joint ALS needs lam > 0"};
        if (!d_F) throw Error{DFACTO_E_INVALID, "NULL argument"};
        for (int m = 0; m < 3; ++m) {
            check_factor(d_F[m], "factor");
            check_align(d_F[m], dtype, "factor");
        }
        Small sw = small_ws(ctx, R);
        float *M = (float *)ws_get(ctx, dfacto_ctx::kM, sizeof(float) * (size_t)max_dim(X) * R);
        // ones row, then the heavy rows' partial systems
        const int64_t nseg = std::max(Y->nseg[0], Y->nseg[1]);
        char *w = (char *)ws_get(ctx, dfacto_ctx::kJoint,
                                 256 + sizeof(double) * (size_t)(nseg * (R * R + R) + 1));
        void *one = ones_row(ctx, R, dtype, w);
        double *part = (double *)(w + 256);
        DF_HIP(hipMemsetAsync(sw.flag, 0, 4 * sizeof(int), ctx->stream));
        ensure_side(ctx);
        for (int n = 0; n < 3; ++n) {
            const int p = (n + 1) % 3, q = (n + 2) % 3;
            const ModeData &md = X->mode[n];
            // Mode n's R x R work needs only the other modes' Grams, final
            // here (and the previous mode's row pass, the last reader of
            // H^-1, is done): it runs on the side stream beside this mode's
            // MTTKRP and is joined before the rows.  Mode 0 first forms the
            // Grams of F[1] and F[2] there.
            DF_HIP(hipEventRecord(ctx->ev_fork, ctx->stream));
            DF_HIP(hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0));
            {
                OnStream on(ctx, ctx->side);
                if (n == 0) {
                    launch_gram(ctx, d_F[1], dtype, X->dims[1], R, sw.G[1]);
                    launch_gram(ctx, d_F[2], dtype, X->dims[2], R, sw.G[2]);
                }
                // users (n = 0), items (n = 1): H for the row systems, and
                // P^-1 for the short rows: (mu H + lam I)^-1 = (H + (lam / mu) I)^-1 / mu;
                // words: C = mu M (mu H + lam I)^-1 = M (H + (lam / mu) I)^-1
                if (n < 2) launch_hadamard(ctx, R, sw.G[p], sw.G[q], 0.0, sw.H[n]);
                if (mu > 0.0)
                    launch_solve(ctx, R, sw.G[p], sw.G[q], lam / mu, sw.Hinv, sw.solve_scratch,
                                 sw.flag + (n < 2 ? 2 : 1));
            }
            DF_HIP(hipEventRecord(ctx->ev_join, ctx->side));
            if (mu > 0.0) launch_mttkrp(ctx, X, n, R, dtype, d_F[md.leaf], d_F[md.mid], M);
            DF_HIP(hipStreamWaitEvent(ctx->stream, ctx->ev_join, 0));
            if (n < 2) {
                // users (n = 0): entries (1, item); items (n = 1): entries (user, 1);
                // without the tensor term P^-1 = I / lam
                const double *Pinv = mu > 0.0 ? sw.Hinv : nullptr;
                const double ws = mu > 0.0 ? 1.0 / mu : 1.0 / lam;
                launch_joint_rows(ctx, Y, n, X->dims[n], n == 0 ? one : d_F[0],
                                  n == 0 ? d_F[1] : one, R, mu > 0.0 ? M : nullptr, sw.H[n], mu,
                                  lam, Pinv, ws, sw.flag + 2, d_F[n], dtype, sw.flag, part);
            } else if (mu > 0.0) {
                launch_rowmap(ctx, M, X->dims[2], R, sw.Hinv, d_F[2], dtype);
            } else {
                DF_HIP(hipMemsetAsync(d_F[2], 0, (size_t)X->dims[2] * R * elem_size(dtype),
                                      ctx->stream));
            }
            launch_gram(ctx, d_F[n], dtype, X->dims[n], R, sw.G[n]);
        }
        int flag = 0;
        DF_HIP(hipMemcpyAsync(&flag, sw.flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        DF_HIP(hipStreamSynchronize(ctx->stream));
        if (flag)
            throw Error{DFACTO_E_NUMERIC, "a joint ALS row system is not numerically positive "
                                          "definite"};
    });
}

dfacto_status dfacto_profile_enable(dfacto_ctx *ctx, int on) {
    return guarded(ctx, [&] {
        ctx->profiling = on != 0;
        ctx->ev_used = 0;
        ctx->prof_bytes = ctx->prof_flops = 0.0;
    });
}

dfacto_status dfacto_profile_read(dfacto_ctx *ctx, int64_t *launches, double *ms, double *bytes,
                                  double *flops) {
    return guarded(ctx, [&] {
        DF_HIP(hipStreamSynchronize(ctx->stream));
        double total = 0.0;
        for (size_t e = 0; e + 1 < ctx->ev_used; e += 2) {
            float t = 0.f;
            DF_HIP(hipEventElapsedTime(&t, ctx->ev_pool[e], ctx->ev_pool[e + 1]));
            total += t;
        }
        if (launches) *launches = (int64_t)(ctx->ev_used / 2);
        if (ms) *ms = total;
        if (bytes) *bytes = ctx->prof_bytes;
        if (flops) *flops = ctx->prof_flops;
        ctx->ev_used = 0;
        ctx->prof_bytes = ctx->prof_flops = 0.0;
    });
}

}  // extern "C"
