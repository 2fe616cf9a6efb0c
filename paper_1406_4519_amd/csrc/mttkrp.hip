// mttkrp.hip -- fused DFacTo MTTKRP for gfx950 (Section 3, Algorithm 1,
// all R rank columns at once).
//
// For output mode n with coordinate roles (root, mid, leaf), DFacTo computes
//   stage 1: value(M^r) <- (Xhat)^T f_leaf_r        (one value per fiber)
//   stage 2: n_r        <- M^r f_mid_r              (one value per root)
// (Lemma 2: column r of X1 (C kr B) is [unvec((X2)^T b_r)]^T c_r; Lemmas 3
// and 4: only nonempty fibers matter and their pattern is fixed).  Here both
// products run in one pass over the mode's stream for all R columns: a group
// of G lanes owns the rank columns (CPL consecutive columns per lane, so a
// factor-row gather is one coalesced 4*CPL-byte load per lane) and walks one
// work chunk of the stream.  The fiber partial P (the paper's value(M^r),
// materialized only in registers) accumulates val * F_leaf[leaf, :]; at the
// next header it is folded into the root accumulator as P * F_mid[mid, :];
// at a new root the accumulator is written out.
//
// Work chunks always start at a header and are balanced in entries, so a
// heavy root is spread over many groups.  A root that begins before the
// chunk (no ROOT bit on the chunk's first header) is written to a per-chunk
// carry slot; the fix-up kernel adds the carries of each such root to the
// owner's row in chunk order.  No floating-point atomics: results are
// deterministic.  The fix-up launch also zero-fills the empty output rows.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace dfacto {
namespace {

constexpr int kBlock = 256;
constexpr int kUnroll = 8;  // stream entries in flight per group
static_assert(kStreamPad >= kUnroll, "stream padding must cover one batch");

// ---- factor-row loads: CPL consecutive columns, widened to FP32 ----------
template <typename T, int CPL>
struct RowLoad;

template <>
struct RowLoad<float, 4> {
    static __device__ __forceinline__ void load(const float *p, float (&v)[4]) {
        const float4 x = *reinterpret_cast<const float4 *>(p);
        v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    }
};
template <>
struct RowLoad<float, 2> {
    static __device__ __forceinline__ void load(const float *p, float (&v)[2]) {
        const float2 x = *reinterpret_cast<const float2 *>(p);
        v[0] = x.x; v[1] = x.y;
    }
};
template <>
struct RowLoad<float, 1> {
    static __device__ __forceinline__ void load(const float *p, float (&v)[1]) { v[0] = *p; }
};

__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

template <>
struct RowLoad<uint16_t, 4> {
    static __device__ __forceinline__ void load(const uint16_t *p, float (&v)[4]) {
        const uint2 x = *reinterpret_cast<const uint2 *>(p);
        v[0] = bf16_lo(x.x); v[1] = bf16_hi(x.x); v[2] = bf16_lo(x.y); v[3] = bf16_hi(x.y);
    }
};
template <>
struct RowLoad<uint16_t, 2> {
    static __device__ __forceinline__ void load(const uint16_t *p, float (&v)[2]) {
        const uint32_t x = *reinterpret_cast<const uint32_t *>(p);
        v[0] = bf16_lo(x); v[1] = bf16_hi(x);
    }
};
template <>
struct RowLoad<uint16_t, 1> {
    static __device__ __forceinline__ void load(const uint16_t *p, float (&v)[1]) {
        v[0] = __uint_as_float((uint32_t)(*p) << 16);
    }
};

template <int CPL>
__device__ __forceinline__ void store_vec(float *p, const float (&v)[CPL]) {
    if constexpr (CPL == 4) {
        *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
    } else if constexpr (CPL == 2) {
        *reinterpret_cast<float2 *>(p) = make_float2(v[0], v[1]);
    } else {
        p[0] = v[0];
    }
}

template <int CPL>
__device__ __forceinline__ void load_f32(const float *p, float (&v)[CPL]) {
    RowLoad<float, CPL>::load(p, v);
}

// ---- main kernel ---------------------------------------------------------
template <typename T, int CPL, int G, int NCH>
__global__ __launch_bounds__(kBlock) void k_mttkrp(
    const uint2 *__restrict__ st, const uint32_t *__restrict__ cstart, uint32_t nchunk,
    const T *__restrict__ Fleaf, const T *__restrict__ Fmid, int R, float *__restrict__ out,
    float *__restrict__ carry) {
    const uint32_t gid = (blockIdx.x * (uint32_t)kBlock + threadIdx.x) / G;
    const int lane = threadIdx.x % G;
    if (gid >= nchunk) return;
    const uint32_t cs = cstart[gid], ce = cstart[gid + 1];
    if (cs >= ce) return;

    int col[NCH];
    bool act[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        col[c] = (c * G + lane) * CPL;
        act[c] = col[c] < R;
    }
    float acc[NCH][CPL], p[NCH][CPL], mrow[NCH][CPL];
    const uint2 h0 = st[cs];
    uint32_t row = h0.y;
    bool cont = !(h0.x & kRootBit);
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
#pragma unroll
        for (int q = 0; q < CPL; ++q) acc[c][q] = p[c][q] = mrow[c][q] = 0.f;
        if (act[c]) RowLoad<T, CPL>::load(Fmid + (size_t)(h0.x & kIdxMask) * R + col[c], mrow[c]);
    }

    auto flush = [&](uint32_t r_out, bool is_cont) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            if (!act[c]) continue;
            float *dst = is_cont ? carry + (size_t)gid * R + col[c] : out + (size_t)r_out * R + col[c];
            store_vec<CPL>(dst, acc[c]);
        }
    };

    for (uint32_t e = cs + 1; e < ce; e += kUnroll) {
        uint2 w[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) w[u] = st[e + u];  // padded stream: always in bounds
        float g[kUnroll][NCH][CPL];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const bool valid = e + u < ce;
            const T *base = (w[u].x & kHdrBit) ? Fmid : Fleaf;
            const size_t off = (size_t)(w[u].x & kIdxMask) * R;
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                if (valid && act[c]) {
                    RowLoad<T, CPL>::load(base + off + col[c], g[u][c]);
                } else {
#pragma unroll
                    for (int q = 0; q < CPL; ++q) g[u][c][q] = 0.f;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (e + u >= ce) break;
            if (w[u].x & kHdrBit) {
                // end of a fiber segment: stage 2 for the finished partial
#pragma unroll
                for (int c = 0; c < NCH; ++c)
#pragma unroll
                    for (int q = 0; q < CPL; ++q) {
                        acc[c][q] = fmaf(p[c][q], mrow[c][q], acc[c][q]);
                        p[c][q] = 0.f;
                        mrow[c][q] = g[u][c][q];
                    }
                if (w[u].x & kRootBit) {
                    flush(row, cont);
#pragma unroll
                    for (int c = 0; c < NCH; ++c)
#pragma unroll
                        for (int q = 0; q < CPL; ++q) acc[c][q] = 0.f;
                    cont = false;
                    row = w[u].y;
                }
            } else {
                // stage 1: accumulate the fiber partial
                const float v = __uint_as_float(w[u].y);
#pragma unroll
                for (int c = 0; c < NCH; ++c)
#pragma unroll
                    for (int q = 0; q < CPL; ++q) p[c][q] = fmaf(v, g[u][c][q], p[c][q]);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int q = 0; q < CPL; ++q) acc[c][q] = fmaf(p[c][q], mrow[c][q], acc[c][q]);
    flush(row, cont);
}

// ---- fix-up: continuation carries and empty rows --------------------------
template <int CPL, int G, int NCH>
__global__ __launch_bounds__(kBlock) void k_mttkrp_fixup(
    const uint2 *__restrict__ st, const uint32_t *__restrict__ cstart, uint32_t nchunk,
    const float *__restrict__ carry, int R, float *__restrict__ out,
    const uint32_t *__restrict__ empty_rows, uint32_t nempty, uint32_t nempty_groups) {
    const uint32_t gid = (blockIdx.x * (uint32_t)kBlock + threadIdx.x) / G;
    const int lane = threadIdx.x % G;
    int col[NCH];
    bool act[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        col[c] = (c * G + lane) * CPL;
        act[c] = col[c] < R;
    }
    if (gid < nchunk) {
        const uint32_t cs = cstart[gid];
        if (cs >= cstart[gid + 1]) return;
        const uint2 h = st[cs];
        if (h.x & kRootBit) return;  // chunk starts its own root: nothing carried
        if (gid > 0) {
            const uint2 hp = st[cstart[gid - 1]];
            if (!(hp.x & kRootBit) && hp.y == h.y) return;  // not the first carry of the run
        }
        const uint32_t row = h.y;
        float acc[NCH][CPL];
#pragma unroll
        for (int c = 0; c < NCH; ++c)
            if (act[c]) load_f32<CPL>(out + (size_t)row * R + col[c], acc[c]);
        for (uint32_t ch = gid; ch < nchunk; ++ch) {
            const uint32_t a = cstart[ch];
            if (a >= cstart[ch + 1]) break;
            const uint2 hc = st[a];
            if ((hc.x & kRootBit) || hc.y != row) break;
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                if (!act[c]) continue;
                float v[CPL];
                load_f32<CPL>(carry + (size_t)ch * R + col[c], v);
#pragma unroll
                for (int q = 0; q < CPL; ++q) acc[c][q] += v[q];
            }
        }
#pragma unroll
        for (int c = 0; c < NCH; ++c)
            if (act[c]) store_vec<CPL>(out + (size_t)row * R + col[c], acc[c]);
    } else {
        const uint32_t eg = gid - nchunk;
        if (eg >= nempty_groups) return;
        float z[CPL];
#pragma unroll
        for (int q = 0; q < CPL; ++q) z[q] = 0.f;
        for (uint32_t r = eg; r < nempty; r += nempty_groups) {
            const uint32_t row = empty_rows[r];
#pragma unroll
            for (int c = 0; c < NCH; ++c)
                if (act[c]) store_vec<CPL>(out + (size_t)row * R + col[c], z);
        }
    }
}

// ---- dispatch --------------------------------------------------------------
struct Shape {
    int cpl, g, nch;
};

Shape pick_shape(int R, bool aligned4, bool aligned2) {
    int cpl = 1;
    if (R % 4 == 0 && aligned4) cpl = 4;
    else if (R % 2 == 0 && aligned2) cpl = 2;
    const int lanes = (R + cpl - 1) / cpl;
    if (lanes <= 64) {
        int g = 2;
        while (g < lanes) g <<= 1;
        return {cpl, g, 1};
    }
    int nch = (lanes + 63) / 64;
    nch = nch <= 2 ? 2 : 4;
    return {cpl, 64, nch};
}

template <typename T, int CPL, int G, int NCH>
void run(dfacto_ctx *ctx, const ModeData &md, int R, const void *Fleaf, const void *Fmid,
         float *out) {
    hipStream_t s = ctx->stream;
    const uint32_t nchunk = (uint32_t)md.nchunk;
    float *carry = (float *)ws_get(ctx, dfacto_ctx::kCarry,
                                   sizeof(float) * (size_t)std::max<int64_t>(md.nchunk, 1) * R);
    constexpr int gpb = kBlock / G;  // groups per block
    if (nchunk > 0) {
        const unsigned blocks = (nchunk + gpb - 1) / gpb;
        prof_mark(ctx);
        hipLaunchKernelGGL((k_mttkrp<T, CPL, G, NCH>), dim3(blocks), dim3(kBlock), 0, s,
                           md.stream, md.chunk_start, nchunk, (const T *)Fleaf, (const T *)Fmid, R,
                           out, carry);
        prof_mark(ctx);
    }
    const uint32_t nempty = (uint32_t)md.nempty;
    const uint32_t egroups = nempty == 0 ? 0u : std::min<uint32_t>(nempty, 65536u);
    const uint64_t groups = (uint64_t)nchunk + egroups;
    if (groups > 0) {
        const unsigned blocks = (unsigned)((groups + gpb - 1) / gpb);
        hipLaunchKernelGGL((k_mttkrp_fixup<CPL, G, NCH>), dim3(blocks), dim3(kBlock), 0, s,
                           md.stream, md.chunk_start, nchunk, carry, R, out, md.empty_rows, nempty,
                           egroups);
    }
    DF_HIP(hipGetLastError());
}

template <typename T, int CPL>
void run_cpl(dfacto_ctx *ctx, const ModeData &md, int R, const Shape &sh, const void *Fl,
             const void *Fm, float *out) {
    if (sh.nch == 1) {
        switch (sh.g) {
            case 2: return run<T, CPL, 2, 1>(ctx, md, R, Fl, Fm, out);
            case 4: return run<T, CPL, 4, 1>(ctx, md, R, Fl, Fm, out);
            case 8: return run<T, CPL, 8, 1>(ctx, md, R, Fl, Fm, out);
            case 16: return run<T, CPL, 16, 1>(ctx, md, R, Fl, Fm, out);
            case 32: return run<T, CPL, 32, 1>(ctx, md, R, Fl, Fm, out);
            default: return run<T, CPL, 64, 1>(ctx, md, R, Fl, Fm, out);
        }
    }
    if constexpr (CPL < 4) {
        if (sh.nch == 2) return run<T, CPL, 64, 2>(ctx, md, R, Fl, Fm, out);
    }
    if constexpr (CPL == 1) {
        return run<T, CPL, 64, 4>(ctx, md, R, Fl, Fm, out);
    }
    throw Error{DFACTO_E_UNSUPPORTED, "no MTTKRP kernel for this rank"};
}

}  // namespace

void launch_mttkrp(dfacto_ctx *ctx, const dfacto_tensor *t, int mode, int R, dfacto_dtype dtype,
                   const void *Fleaf, const void *Fmid, float *out) {
    const ModeData &md = t->mode[mode];
    if (ctx->profiling && md.nchunk > 0) {
        const double sf = dtype == DFACTO_BF16 ? 2.0 : 4.0;
        ctx->prof_bytes += 8.0 * (double)t->nnz + 8.0 * (double)md.nfib + 8.0 * (double)md.nroot +
                           4.0 * (double)t->dims[md.root] * R +
                           sf * (double)(t->dims[md.leaf] + t->dims[md.mid]) * R;
        ctx->prof_flops += 2.0 * R * (double)(t->nnz + md.nfib);
    }
    const size_t es = dtype == DFACTO_BF16 ? 2 : 4;
    auto al = [&](size_t a) {
        return ((uintptr_t)Fleaf % a == 0) && ((uintptr_t)Fmid % a == 0) &&
               ((uintptr_t)out % (a * 4 / es) == 0);
    };
    const Shape sh = pick_shape(R, al(4 * es), al(2 * es));
    if (dtype == DFACTO_F32) {
        switch (sh.cpl) {
            case 4: return run_cpl<float, 4>(ctx, md, R, sh, Fleaf, Fmid, out);
            case 2: return run_cpl<float, 2>(ctx, md, R, sh, Fleaf, Fmid, out);
            default: return run_cpl<float, 1>(ctx, md, R, sh, Fleaf, Fmid, out);
        }
    }
    switch (sh.cpl) {
        case 4: return run_cpl<uint16_t, 4>(ctx, md, R, sh, Fleaf, Fmid, out);
        case 2: return run_cpl<uint16_t, 2>(ctx, md, R, sh, Fleaf, Fmid, out);
        default: return run_cpl<uint16_t, 1>(ctx, md, R, sh, Fleaf, Fmid, out);
    }
}

}  // namespace dfacto
