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
// carry slot; the fix-up kernels add the carries of each such root to the
// owner's row in a fixed order.  No floating-point atomics: results are
// deterministic.  The fix-up launches also zero-fill the empty output rows.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.hpp"

namespace dfacto {
namespace {

// Tuning knobs (compile-time; the defaults are the measured best).
#ifndef DFACTO_UNROLL
#define DFACTO_UNROLL 8
#endif
#ifndef DFACTO_MAX_CPL
#define DFACTO_MAX_CPL 8
#endif
#ifndef DFACTO_NT_STREAM
#define DFACTO_NT_STREAM 0
#endif
#ifndef DFACTO_SHARE_ENTRIES
#define DFACTO_SHARE_ENTRIES 1
#endif
// At least 5 waves per SIMD: the gathers are latency-bound, and the FP32
// CPL = 4 kernel sits right at the 96-register limit for 5 waves.  Whole-wave
// groups (G = 64) keep the compiler's choice (they would spill).
#ifndef DFACTO_WAVES_PER_EU
#define DFACTO_WAVES_PER_EU 5
#endif
// Eight columns per lane hold twice the gathered data per batch: 4 waves
// per SIMD (128 registers) keep them out of scratch.
#define MTTKRP_OCCUPANCY                                                               \
    __attribute__((amdgpu_waves_per_eu(G <= 32 ? (CPL >= 8 ? 4 : DFACTO_WAVES_PER_EU) : 1)))

constexpr int kBlock = 256;
constexpr int kUnroll = DFACTO_UNROLL;  // stream entries in flight per group
static_assert(kStreamPad >= kUnroll && kStreamPad >= 32, "stream padding must cover a batch");

// f(integral_constant<int, I>) for I = B .. E-1, so I is usable as a constant
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

__device__ __forceinline__ uint2 load_entry(const uint2 *p) {
#if DFACTO_NT_STREAM
    const unsigned long long x =
        __builtin_nontemporal_load(reinterpret_cast<const unsigned long long *>(p));
    return make_uint2((uint32_t)x, (uint32_t)(x >> 32));
#else
    return *p;
#endif
}

__device__ __forceinline__ uint2 load_entry(const DF_GLOBAL uint2 *p) {
#if DFACTO_NT_STREAM
    const unsigned long long x =
        __builtin_nontemporal_load(reinterpret_cast<const DF_GLOBAL unsigned long long *>(p));
    return make_uint2((uint32_t)x, (uint32_t)(x >> 32));
#else
    const df_u2 x = *reinterpret_cast<const DF_GLOBAL df_u2 *>(p);
    return make_uint2(x.x, x.y);
#endif
}

// ---- factor-row loads: CPL consecutive columns, widened to FP32 ----------
template <typename T, int CPL>
struct RowLoad;

template <>
struct RowLoad<float, 4> {
    static __device__ __forceinline__ void load(const float *p, float (&v)[4]) {
        const float4 x = *reinterpret_cast<const float4 *>(p);
        v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    }
    static __device__ __forceinline__ void load(const DF_GLOBAL float *p, float (&v)[4]) {
        const df_f4 x = *reinterpret_cast<const DF_GLOBAL df_f4 *>(p);
        v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    }
};
template <>
struct RowLoad<float, 2> {
    static __device__ __forceinline__ void load(const float *p, float (&v)[2]) {
        const float2 x = *reinterpret_cast<const float2 *>(p);
        v[0] = x.x; v[1] = x.y;
    }
    static __device__ __forceinline__ void load(const DF_GLOBAL float *p, float (&v)[2]) {
        const df_f2 x = *reinterpret_cast<const DF_GLOBAL df_f2 *>(p);
        v[0] = x.x; v[1] = x.y;
    }
};
template <>
struct RowLoad<float, 1> {
    static __device__ __forceinline__ void load(const float *p, float (&v)[1]) { v[0] = *p; }
    static __device__ __forceinline__ void load(const DF_GLOBAL float *p, float (&v)[1]) { v[0] = *p; }
};

template <>
struct RowLoad<float, 8> {
    static __device__ __forceinline__ void load(const float *p, float (&v)[8]) {
        const float4 x = *reinterpret_cast<const float4 *>(p);
        const float4 y = *reinterpret_cast<const float4 *>(p + 4);
        v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
        v[4] = y.x; v[5] = y.y; v[6] = y.z; v[7] = y.w;
    }
    static __device__ __forceinline__ void load(const DF_GLOBAL float *p, float (&v)[8]) {
        const df_f4 x = *reinterpret_cast<const DF_GLOBAL df_f4 *>(p);
        const df_f4 y = *reinterpret_cast<const DF_GLOBAL df_f4 *>(p + 4);
        v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
        v[4] = y.x; v[5] = y.y; v[6] = y.z; v[7] = y.w;
    }
};

__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

template <>
struct RowLoad<uint16_t, 8> {
    static __device__ __forceinline__ void load(const uint16_t *p, float (&v)[8]) {
        const uint4 x = *reinterpret_cast<const uint4 *>(p);
        v[0] = bf16_lo(x.x); v[1] = bf16_hi(x.x); v[2] = bf16_lo(x.y); v[3] = bf16_hi(x.y);
        v[4] = bf16_lo(x.z); v[5] = bf16_hi(x.z); v[6] = bf16_lo(x.w); v[7] = bf16_hi(x.w);
    }
    static __device__ __forceinline__ void load(const DF_GLOBAL uint16_t *p, float (&v)[8]) {
        const df_u4 x = *reinterpret_cast<const DF_GLOBAL df_u4 *>(p);
        v[0] = bf16_lo(x.x); v[1] = bf16_hi(x.x); v[2] = bf16_lo(x.y); v[3] = bf16_hi(x.y);
        v[4] = bf16_lo(x.z); v[5] = bf16_hi(x.z); v[6] = bf16_lo(x.w); v[7] = bf16_hi(x.w);
    }
};
template <>
struct RowLoad<uint16_t, 4> {
    static __device__ __forceinline__ void load(const uint16_t *p, float (&v)[4]) {
        const uint2 x = *reinterpret_cast<const uint2 *>(p);
        v[0] = bf16_lo(x.x); v[1] = bf16_hi(x.x); v[2] = bf16_lo(x.y); v[3] = bf16_hi(x.y);
    }
    static __device__ __forceinline__ void load(const DF_GLOBAL uint16_t *p, float (&v)[4]) {
        const df_u2 x = *reinterpret_cast<const DF_GLOBAL df_u2 *>(p);
        v[0] = bf16_lo(x.x); v[1] = bf16_hi(x.x); v[2] = bf16_lo(x.y); v[3] = bf16_hi(x.y);
    }
};
template <>
struct RowLoad<uint16_t, 2> {
    static __device__ __forceinline__ void load(const uint16_t *p, float (&v)[2]) {
        const uint32_t x = *reinterpret_cast<const uint32_t *>(p);
        v[0] = bf16_lo(x); v[1] = bf16_hi(x);
    }
    static __device__ __forceinline__ void load(const DF_GLOBAL uint16_t *p, float (&v)[2]) {
        const uint32_t x = *reinterpret_cast<const DF_GLOBAL uint32_t *>(p);
        v[0] = bf16_lo(x); v[1] = bf16_hi(x);
    }
};
template <>
struct RowLoad<uint16_t, 1> {
    static __device__ __forceinline__ void load(const uint16_t *p, float (&v)[1]) {
        v[0] = __uint_as_float((uint32_t)(*p) << 16);
    }
    static __device__ __forceinline__ void load(const DF_GLOBAL uint16_t *p, float (&v)[1]) {
        v[0] = __uint_as_float((uint32_t)(*p) << 16);
    }
};

template <int CPL>
__device__ __forceinline__ void store_vec(float *p, const float (&v)[CPL]) {
    if constexpr (CPL == 8) {
        *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
        *reinterpret_cast<float4 *>(p + 4) = make_float4(v[4], v[5], v[6], v[7]);
    } else if constexpr (CPL == 4) {
        *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
    } else if constexpr (CPL == 2) {
        *reinterpret_cast<float2 *>(p) = make_float2(v[0], v[1]);
    } else {
        p[0] = v[0];
    }
}

template <int CPL>
__device__ __forceinline__ void store_vec(DF_GLOBAL float *p, const float (&v)[CPL]) {
    if constexpr (CPL == 8) {
        *reinterpret_cast<DF_GLOBAL df_f4 *>(p) = df_f4{v[0], v[1], v[2], v[3]};
        *reinterpret_cast<DF_GLOBAL df_f4 *>(p + 4) = df_f4{v[4], v[5], v[6], v[7]};
    } else if constexpr (CPL == 4) {
        *reinterpret_cast<DF_GLOBAL df_f4 *>(p) = df_f4{v[0], v[1], v[2], v[3]};
    } else if constexpr (CPL == 2) {
        *reinterpret_cast<DF_GLOBAL df_f2 *>(p) = df_f2{v[0], v[1]};
    } else {
        p[0] = v[0];
    }
}

template <int CPL>
__device__ __forceinline__ void load_f32(const DF_GLOBAL float *p, float (&v)[CPL]) {
    RowLoad<float, CPL>::load(p, v);
}

template <int CPL>
__device__ __forceinline__ void load_f32(const float *p, float (&v)[CPL]) {
    RowLoad<float, CPL>::load(p, v);
}

// ---- factor-row sources ------------------------------------------------------
// load(w, c, v): the row that stream entry w gathers -- the leaf row for a
// nonzero, the mid row for a header -- columns of block c (CPL per lane),
// widened to FP32.  Lanes whose columns lie beyond R read column 0 instead
// (in bounds, never stored), so every gather is issued without a branch and
// the loads of a batch stay in flight together.
// SMALL: every row index is below 2^24, so row offsets are one 24-bit
// multiply (idx * R < 2^32) instead of 64-bit arithmetic.

// Rows straight from the two factor tables in device memory.
template <typename T, int CPL, int NCH, bool SMALL>
struct GlobalRows {
    const DF_GLOBAL T *leafb[NCH], *midb[NCH];
    int R;
    __device__ __forceinline__ GlobalRows(const T *Fleaf, const T *Fmid, int R_, int G, int lane)
        : R(R_) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int col = (c * G + lane) * CPL;
            leafb[c] = gptr(Fleaf) + (col < R ? col : 0);
            midb[c] = gptr(Fmid) + (col < R ? col : 0);
        }
    }
    __device__ __forceinline__ size_t off(uint32_t idx) const {
        if constexpr (SMALL) return (size_t)(uint32_t)__umul24(idx, (uint32_t)R);
        else return (size_t)idx * (size_t)R;
    }
    __device__ __forceinline__ void load(const uint2 &w, int c, float (&v)[CPL]) const {
        const bool hdr = (int32_t)w.x < 0;  // kHdrBit is the sign bit
        RowLoad<T, CPL>::load((hdr ? midb[c] : leafb[c]) + off(w.x & kIdxMask), v);
    }
};

// CPL elements of T at byte offset `off` of a buffer resource; an offset
// past the buffer's end loads zeros and makes no memory request.
template <typename T, int CPL>
struct BufLoad;
template <>
struct BufLoad<float, 4> {
    static __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, uint32_t off,
                                                float (&v)[4]) {
        const auto x = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
        v[0] = __uint_as_float(x[0]); v[1] = __uint_as_float(x[1]);
        v[2] = __uint_as_float(x[2]); v[3] = __uint_as_float(x[3]);
    }
};
template <>
struct BufLoad<float, 2> {
    static __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, uint32_t off,
                                                float (&v)[2]) {
        const auto x = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
        v[0] = __uint_as_float(x[0]); v[1] = __uint_as_float(x[1]);
    }
};
template <>
struct BufLoad<float, 1> {
    static __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, uint32_t off,
                                                float (&v)[1]) {
        v[0] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    }
};
template <>
struct BufLoad<float, 8> {  // two 16-byte loads
    static __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, uint32_t off,
                                                float (&v)[8]) {
        const auto x = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
        const auto y = __builtin_amdgcn_raw_buffer_load_b128(r, off + 16u, 0, 0);
        v[0] = __uint_as_float(x[0]); v[1] = __uint_as_float(x[1]);
        v[2] = __uint_as_float(x[2]); v[3] = __uint_as_float(x[3]);
        v[4] = __uint_as_float(y[0]); v[5] = __uint_as_float(y[1]);
        v[6] = __uint_as_float(y[2]); v[7] = __uint_as_float(y[3]);
    }
};
template <>
struct BufLoad<uint16_t, 8> {
    static __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, uint32_t off,
                                                float (&v)[8]) {
        const auto x = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
        v[0] = bf16_lo(x[0]); v[1] = bf16_hi(x[0]); v[2] = bf16_lo(x[1]); v[3] = bf16_hi(x[1]);
        v[4] = bf16_lo(x[2]); v[5] = bf16_hi(x[2]); v[6] = bf16_lo(x[3]); v[7] = bf16_hi(x[3]);
    }
};
template <>
struct BufLoad<uint16_t, 4> {
    static __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, uint32_t off,
                                                float (&v)[4]) {
        const auto x = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
        v[0] = bf16_lo(x[0]); v[1] = bf16_hi(x[0]); v[2] = bf16_lo(x[1]); v[3] = bf16_hi(x[1]);
    }
};
template <>
struct BufLoad<uint16_t, 2> {
    static __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, uint32_t off,
                                                float (&v)[2]) {
        const uint32_t x = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
        v[0] = bf16_lo(x); v[1] = bf16_hi(x);
    }
};
template <>
struct BufLoad<uint16_t, 1> {
    static __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, uint32_t off,
                                                float (&v)[1]) {
        v[0] = __uint_as_float((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0) << 16);
    }
};

// ---- main kernel ---------------------------------------------------------
// One work chunk (gid) per lane group of G lanes (lane = 0 .. G-1), its
// factor rows from `src`.
// RES: the residual form used by the joint model's ratings term: each
// nonzero's value x becomes x - xhat with xhat = sum_r F_root[root, r]
// F_mid[mid, r] F_leaf[leaf, r] (the CP model at that entry), so the output
// is the MTTKRP of the residual restricted to the stored entries.  The dot
// product is reduced across the group's lanes by xor shuffles (every lane
// ends with the same sum: each step adds two commuted operands).
template <typename T, int CPL, int G, int NCH, bool SMALL, bool RES = false, class Src>
__device__ __forceinline__ void mttkrp_chunk(const uint2 *__restrict__ st_,
                                             const uint32_t *__restrict__ cstart, uint32_t nchunk,
                                             const Src &src, int R,
                                             float *__restrict__ out_, float *__restrict__ carry_,
                                             uint32_t gid, int lane,
                                             const T *__restrict__ Froot = nullptr) {
    if (gid >= nchunk) return;
    const uint32_t cs = gptr(cstart)[gid], ce = gptr(cstart)[gid + 1];
    if (cs >= ce) return;
    const DF_GLOBAL uint2 *__restrict__ st = gptr(st_);
    DF_GLOBAL float *__restrict__ out = gptr(out_);
    DF_GLOBAL float *__restrict__ carry = gptr(carry_);

    int col[NCH];
    bool act[NCH];
    const DF_GLOBAL T *rootb[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        col[c] = (c * G + lane) * CPL;
        act[c] = col[c] < R;
        rootb[c] = RES ? gptr(Froot) + (act[c] ? col[c] : 0) : nullptr;
    }
    auto row_off = [&](uint32_t idx) -> size_t {
        if constexpr (SMALL) return (size_t)(uint32_t)__umul24(idx, (uint32_t)R);
        else return (size_t)idx * (size_t)R;
    };
    float acc[NCH][CPL], p[NCH][CPL], mrow[NCH][CPL];
    float rrow[RES ? NCH : 1][CPL];  // the root's factor row (RES only)
    const uint2 h0 = load_entry(st + cs);
    uint32_t row = h0.y;
    bool cont = !(h0.x & kRootBit);
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
#pragma unroll
        for (int q = 0; q < CPL; ++q) acc[c][q] = p[c][q] = 0.f;
        src.load(h0, c, mrow[c]);  // h0 is a header: its mid row
        if constexpr (RES) RowLoad<T, CPL>::load(rootb[c] + row_off(row), rrow[c]);
    }

    auto flush = [&](uint32_t r_out, bool is_cont) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            if (!act[c]) continue;
            DF_GLOBAL float *dst =
                is_cont ? carry + (size_t)gid * R + col[c] : out + row_off(r_out) + col[c];
            store_vec<CPL>(dst, acc[c]);
        }
    };

    // Gathers of one batch: every entry's factor row, without branches.
    // Entries at or past the chunk end are still valid stream entries (the
    // next chunk's, or the padding sentinels with index 0), so these loads
    // are in bounds; their values are ignored.
    auto gather = [&](const uint2 (&w)[kUnroll], float (&g)[kUnroll][NCH][CPL]) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int c = 0; c < NCH; ++c) src.load(w[u], c, g[u][c]);
    };
    // One stream entry, without data-dependent branches except the (rarer)
    // write of a finished output row.  A header closes the fiber segment --
    // stage 2 of Algorithm 1, acc += P * F_mid[mid] -- and opens the next
    // one (P = 0, new mid row); a nonzero accumulates stage 1, P += x *
    // F_leaf[leaf].
    auto step = [&](const uint2 &w, const float (&g)[NCH][CPL]) {
        const bool hdr = (int32_t)w.x < 0;
        float v = hdr ? 0.f : __uint_as_float(w.y);
        if constexpr (RES) {
            float part = 0.f;
#pragma unroll
            for (int c = 0; c < NCH; ++c)
#pragma unroll
                for (int q = 0; q < CPL; ++q)
                    part = fmaf(act[c] ? rrow[c][q] * mrow[c][q] : 0.f, g[c][q], part);
#pragma unroll
            for (int o = G / 2; o > 0; o >>= 1) part += __shfl_xor(part, o, G);
            v = hdr ? 0.f : v - part;
        }
#pragma unroll
        for (int c = 0; c < NCH; ++c)
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
                const float a2 = fmaf(p[c][q], mrow[c][q], acc[c][q]);
                acc[c][q] = hdr ? a2 : acc[c][q];
                p[c][q] = fmaf(v, g[c][q], hdr ? 0.f : p[c][q]);
                mrow[c][q] = hdr ? g[c][q] : mrow[c][q];
            }
        if (hdr && (w.x & kRootBit)) {
            flush(row, cont);
#pragma unroll
            for (int c = 0; c < NCH; ++c)
#pragma unroll
                for (int q = 0; q < CPL; ++q) acc[c][q] = 0.f;
            cont = false;
            row = w.y;
            if constexpr (RES) {
#pragma unroll
                for (int c = 0; c < NCH; ++c) RowLoad<T, CPL>::load(rootb[c] + row_off(row), rrow[c]);
            }
        }
    };

    // Stream entries of a batch.  With groups of at most 32 lanes, lane l
    // loads only entries l, l + G, ... of the batch (8 bytes each) and the
    // group shares them through ds_swizzle (the LDS crossbar), so the vector
    // memory path carries each entry once instead of once per lane.  A
    // 64-lane group is the whole wave and loads the batch directly.
    constexpr bool kShare = G <= 32 && DFACTO_SHARE_ENTRIES;
    constexpr int KL = kShare ? (kUnroll + G - 1) / G : kUnroll;  // entries held per lane
    auto load_batch = [&](uint32_t at, uint2 (&wl)[KL]) {
#pragma unroll
        for (int k = 0; k < KL; ++k)
            wl[k] = kShare ? load_entry(st + at + lane + G * k) : load_entry(st + at + k);
    };
    auto expand = [&](const uint2 (&wl)[KL], uint2 (&w)[kUnroll]) {
        static_for<0, kUnroll>([&](auto uc) {
            constexpr int u = decltype(uc)::value;
            if constexpr (kShare) {
                // bit-mask swizzle: source lane = (lane & ~(G-1)) | (u % G), within 32 lanes
                constexpr int pat = (0x1F & ~(G - 1)) | ((u % G) << 5);
                w[u].x = (uint32_t)__builtin_amdgcn_ds_swizzle((int)wl[u / G].x, pat);
                w[u].y = (uint32_t)__builtin_amdgcn_ds_swizzle((int)wl[u / G].y, pat);
            } else {
                w[u] = wl[u];
            }
        });
    };

    // Full batches.  The next batch's entries are requested right after the
    // current batch's gathers, so their latency overlaps the gathers.  The
    // stream padding (>= 64 entries) keeps the look-ahead in bounds.
    uint32_t e = cs + 1;
    uint2 wn[KL];
    load_batch(e, wn);
    for (; e + kUnroll <= ce; e += kUnroll) {
        uint2 w[kUnroll];
        expand(wn, w);
        float g[kUnroll][NCH][CPL];
        gather(w, g);
        load_batch(e + kUnroll, wn);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) step(w[u], g[u]);
    }
    // Last, partial batch (fewer than kUnroll entries left).
    if (e < ce) {
        uint2 w[kUnroll];
        expand(wn, w);
        float g[kUnroll][NCH][CPL];
        gather(w, g);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            if (e + u < ce) step(w[u], g[u]);
    }
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int q = 0; q < CPL; ++q) acc[c][q] = fmaf(p[c][q], mrow[c][q], acc[c][q]);
    flush(row, cont);
}

template <typename T, int CPL, int G, int NCH, bool SMALL>
__global__ __launch_bounds__(kBlock) MTTKRP_OCCUPANCY void k_mttkrp(
    const uint2 *__restrict__ st, const uint32_t *__restrict__ cstart, uint32_t nchunk,
    const T *__restrict__ Fleaf, const T *__restrict__ Fmid, int R, float *__restrict__ out,
    float *__restrict__ carry) {
    const int lane = threadIdx.x % G;
    const GlobalRows<T, CPL, NCH, SMALL> src(Fleaf, Fmid, R, G, lane);
    mttkrp_chunk<T, CPL, G, NCH, SMALL>(st, cstart, nchunk, src, R, out, carry,
                                        (blockIdx.x * (uint32_t)kBlock + threadIdx.x) / G, lane);
}

template <typename T, int CPL, int G, int NCH, bool SMALL>
__global__ __launch_bounds__(kBlock) void k_mttkrp_res(
    const uint2 *__restrict__ st, const uint32_t *__restrict__ cstart, uint32_t nchunk,
    const T *__restrict__ Fleaf, const T *__restrict__ Fmid, const T *__restrict__ Froot, int R,
    float *__restrict__ out, float *__restrict__ carry) {
    const int lane = threadIdx.x % G;
    const GlobalRows<T, CPL, NCH, SMALL> src(Fleaf, Fmid, R, G, lane);
    mttkrp_chunk<T, CPL, G, NCH, SMALL, true>(st, cstart, nchunk, src, R, out, carry,
                                              (blockIdx.x * (uint32_t)kBlock + threadIdx.x) / G,
                                              lane, Froot);
}

// Grouped MTTKRP over many tensors of one kernel shape: a persistent grid
// walks the work items (tensor, first chunk of kBlock / G * kper
// consecutive chunks) in a fixed order, item blockIdx.x, blockIdx.x +
// gridDim.x, ...; each lane group takes kper consecutive chunks of its item
// in turn.  Every chunk writes its own rows and carry, so the grid, the
// shape and kper change no result.
template <typename T, int CPL, int G, int NCH, bool SMALL>
__global__ __launch_bounds__(kBlock) MTTKRP_OCCUPANCY void k_mttkrp_group(
    const GroupMttkrp *__restrict__ desc, const uint2 *__restrict__ items, uint32_t nitems,
    uint32_t kper) {
    const int lane = threadIdx.x % G;
    if (kper == 1) {  // the common form, without the inner loop
        for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
            const uint2 w = items[it];
            const GroupMttkrp &d = desc[w.x];
            const GlobalRows<T, CPL, NCH, SMALL> src((const T *)d.Fleaf, (const T *)d.Fmid, d.R,
                                                     G, lane);
            mttkrp_chunk<T, CPL, G, NCH, SMALL>(d.stream, d.chunk_start, d.nchunk, src, d.R,
                                                d.out, d.carry, w.y + threadIdx.x / G, lane);
        }
        return;
    }
    const uint32_t first = (threadIdx.x / G) * kper;
    for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const uint2 w = items[it];
        const GroupMttkrp &d = desc[w.x];
        const GlobalRows<T, CPL, NCH, SMALL> src((const T *)d.Fleaf, (const T *)d.Fmid, d.R, G,
                                                 lane);
        for (uint32_t q = 0; q < kper; ++q)
            mttkrp_chunk<T, CPL, G, NCH, SMALL>(d.stream, d.chunk_start, d.nchunk, src, d.R,
                                                d.out, d.carry, w.y + first + q, lane);
    }
}

// ---- gather ceiling --------------------------------------------------------
// The main kernel's memory requests without its arithmetic: the same work
// chunks, lane groups, batches of kUnroll entries (shared through
// ds_swizzle) and row loads, but every gathered row is only summed.  PAT
// selects the row that an entry gathers:
//   0  the entry's own row (leaf for a nonzero, mid for a header): the
//      MTTKRP's exact request sequence;
//   1  a row drawn uniformly from the same table (hash of the position);
//   2  a row among the table's first 4096 (a working set that stays in L2);
//   3  none: the stream is read, nothing is gathered.
// Each lane writes its sum to sink[gid * G + lane], so nothing is elided.
__device__ __forceinline__ uint32_t probe_hash(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

constexpr int kProbeLdsRows = 128, kProbeLdsRowElems = 64;

template <typename T, int CPL, int G, bool SMALL, int PAT>
__global__ __launch_bounds__(kBlock) MTTKRP_OCCUPANCY void k_gather_probe(
    const uint2 *__restrict__ st, const uint32_t *__restrict__ cstart, uint32_t nchunk,
    const T *__restrict__ Fleaf, const T *__restrict__ Fmid, int R, uint32_t nleaf,
    uint32_t nmid, float *__restrict__ sink) {
    const uint32_t gid0 = (blockIdx.x * (uint32_t)kBlock + threadIdx.x) / G;
    const int lane = threadIdx.x % G;
    // groups past the last chunk walk an empty range (they still take part
    // in the block's barrier)
    const uint32_t gid = gid0 < nchunk ? gid0 : nchunk;
    const uint32_t cs = cstart[gid], ce = gid0 < nchunk ? cstart[gid + 1] : cs;
    const int col = lane * CPL;
    const bool act = col < R;
    const T *leafb = Fleaf + (act ? col : 0), *midb = Fmid + (act ? col : 0);
    auto row_off = [&](uint32_t idx) -> size_t {
        if constexpr (SMALL) return (size_t)(uint32_t)__umul24(idx, (uint32_t)R);
        else return (size_t)idx * (size_t)R;
    };
    float acc[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) acc[q] = 0.f;
    // PAT 5, 8, 9: rows read from an LDS table (kProbeLdsRows rows)
    constexpr bool kLds = PAT == 5 || PAT == 8 || PAT == 9;
    __shared__ T lds_rows[kLds ? kProbeLdsRows * kProbeLdsRowElems : 1];
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void *)Fleaf, (short)0, (int)((uint64_t)nleaf * R * sizeof(T) < 0xFFFFFF00ull
                                            ? (uint64_t)nleaf * R * sizeof(T)
                                            : 0xFFFFFF00ull),
        0x00020000);
    if constexpr (kLds) {
        const uint64_t have = (uint64_t)nleaf * (uint64_t)R;
        const uint32_t nfill = have < (uint64_t)kProbeLdsRowElems ? (uint32_t)have
                                                                   : (uint32_t)kProbeLdsRowElems;
        for (int x = threadIdx.x; x < kProbeLdsRows * kProbeLdsRowElems; x += kBlock)
            lds_rows[x] = Fleaf[(uint32_t)x % nfill];
        __syncthreads();
    }
    constexpr bool kShare = G <= 32 && DFACTO_SHARE_ENTRIES;
    constexpr int KL = kShare ? (kUnroll + G - 1) / G : kUnroll;
    auto load_batch = [&](uint32_t at, uint2 (&wl)[KL]) {
#pragma unroll
        for (int k = 0; k < KL; ++k)
            wl[k] = kShare ? load_entry(st + at + lane + G * k) : load_entry(st + at + k);
    };
    auto expand = [&](const uint2 (&wl)[KL], uint2 (&w)[kUnroll]) {
        static_for<0, kUnroll>([&](auto uc) {
            constexpr int u = decltype(uc)::value;
            if constexpr (kShare) {
                constexpr int pat = (0x1F & ~(G - 1)) | ((u % G) << 5);
                w[u].x = (uint32_t)__builtin_amdgcn_ds_swizzle((int)wl[u / G].x, pat);
                w[u].y = (uint32_t)__builtin_amdgcn_ds_swizzle((int)wl[u / G].y, pat);
            } else {
                w[u] = wl[u];
            }
        });
    };
    uint2 wn[KL];
    load_batch(cs, wn);
    for (uint32_t e = cs; e < ce; e += kUnroll) {
        uint2 w[kUnroll];
        expand(wn, w);
        load_batch(e + kUnroll, wn);
        float g[kUnroll][CPL];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const bool hdr = (int32_t)w[u].x < 0;
            if constexpr (PAT == 3) {
#pragma unroll
                for (int q = 0; q < CPL; ++q) g[u][q] = __uint_as_float(w[u].y & 0x3F7FFFFFu);
            } else if constexpr (PAT == 5) {
                const uint32_t h = probe_hash(e + u) & (kProbeLdsRows - 1);
                RowLoad<T, CPL>::load(lds_rows + h * (kProbeLdsRowElems) + (act ? col : 0), g[u]);
            } else if constexpr (PAT >= 6) {
                // buffer loads of leaf rows: 6 every offset out of range; 7 the
                // entry's own row (mid index taken modulo the leaf rows); 8 half
                // of the entries (a hash bit) from the LDS table, the other
                // half own rows, split by a branch; 9 the same half split
                // without a branch (out-of-range buffer load + LDS row 0)
                const uint32_t idx = (w[u].x & kIdxMask) % nleaf;
                const uint32_t boff = (uint32_t)(idx * (uint32_t)R + (act ? col : 0)) * sizeof(T);
                const bool lhot = (probe_hash(e + u) & 1u) != 0;
                const uint32_t h = probe_hash(e + u) >> 25;  // < 128 rows
                if constexpr (PAT == 6) {
                    BufLoad<T, CPL>::load(rsrc, 0xFFFFFF00u, g[u]);
                } else if constexpr (PAT == 7) {
                    BufLoad<T, CPL>::load(rsrc, boff, g[u]);
                } else if constexpr (PAT == 8) {
                    if (lhot)
                        RowLoad<T, CPL>::load(lds_rows + h * kProbeLdsRowElems + (act ? col : 0),
                                              g[u]);
                    else
                        BufLoad<T, CPL>::load(rsrc, boff, g[u]);
                } else {
                    float gv[CPL], lv[CPL];
                    BufLoad<T, CPL>::load(rsrc, lhot ? 0xFFFFFF00u : boff, gv);
                    RowLoad<T, CPL>::load(lds_rows + (lhot ? h : 0u) * kProbeLdsRowElems +
                                              (act ? col : 0),
                                          lv);
#pragma unroll
                    for (int q = 0; q < CPL; ++q) g[u][q] = lhot ? lv[q] : gv[q];
                }
            } else {
                uint32_t idx;
                if constexpr (PAT == 0) {
                    idx = w[u].x & kIdxMask;
                } else {
                    const uint32_t n = hdr ? nmid : nleaf;
                    const uint32_t h = probe_hash(e + u);
                    const uint32_t lim = PAT == 2 ? 4096u : 32u;
                    idx = PAT == 1 ? (uint32_t)(((uint64_t)h * n) >> 32)
                                   : (h & (lim - 1)) % (n < lim ? n : lim);
                }
                RowLoad<T, CPL>::load((hdr ? midb : leafb) + row_off(idx), g[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int q = 0; q < CPL; ++q) acc[q] += (e + u < ce) ? g[u][q] : 0.f;
    }
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < CPL; ++q) s += acc[q];
    if (gid0 < nchunk) sink[(size_t)gid * G + lane] = s;
}

// ---- fix-up: carries of split rows, and empty rows ------------------------
// out[row] += carry[c0] + ... + carry[c0 + n - 1], in chunk order (one lane
// group; col/act are the lane's column blocks)
template <int CPL, int NCH>
__device__ __forceinline__ void add_run(const float *__restrict__ carry_, int R,
                                        float *__restrict__ out_, uint32_t row, uint32_t c0,
                                        uint32_t n, const int (&col)[NCH], const bool (&act)[NCH]) {
    const DF_GLOBAL float *__restrict__ carry = gptr(carry_);
    DF_GLOBAL float *__restrict__ out = gptr(out_);
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        if (!act[c]) continue;
        float acc[CPL];
        load_f32<CPL>(out + (size_t)row * R + col[c], acc);
        for (uint32_t k = 0; k < n; ++k) {
            float v[CPL];
            load_f32<CPL>(carry + (size_t)(c0 + k) * R + col[c], v);
#pragma unroll
            for (int q = 0; q < CPL; ++q) acc[q] += v[q];
        }
        store_vec<CPL>(out + (size_t)row * R + col[c], acc);
    }
}

template <int CPL, int NCH>
__device__ __forceinline__ void zero_row(float *__restrict__ out_, int R, uint32_t row,
                                         const int (&col)[NCH], const bool (&act)[NCH]) {
    DF_GLOBAL float *__restrict__ out = gptr(out_);
    float z[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) z[q] = 0.f;
#pragma unroll
    for (int c = 0; c < NCH; ++c)
        if (act[c]) store_vec<CPL>(out + (size_t)row * R + col[c], z);
}

// Short runs: one lane group per run adds its <= kShortRun carries in chunk
// order; the groups after the runs zero-fill the empty output rows.
template <int CPL, int G, int NCH>
__device__ __forceinline__ void short_runs(uint32_t gid, const uint32_t *__restrict__ runs,
                                           uint32_t nruns, const float *__restrict__ carry, int R,
                                           float *__restrict__ out,
                                           const uint32_t *__restrict__ empty_rows,
                                           uint32_t nempty, uint32_t nempty_groups) {
    const int lane = threadIdx.x % G;
    int col[NCH];
    bool act[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        col[c] = (c * G + lane) * CPL;
        act[c] = col[c] < R;
    }
    if (gid < nruns) {
        add_run<CPL, NCH>(carry, R, out, runs[3 * gid], runs[3 * gid + 1], runs[3 * gid + 2], col,
                          act);
        return;
    }
    const uint32_t eg = gid - nruns;
    if (eg >= nempty_groups) return;
    for (uint32_t r = eg; r < nempty; r += nempty_groups)
        zero_row<CPL, NCH>(out, R, empty_rows[r], col, act);
}

// Long runs: one workgroup per run; kBlock / G slices each sum a strided
// subset of the carries, then a fixed-order tree over the slices (so the
// result is deterministic) is added to the row.
constexpr int kLongBlock = 1024;

template <int CPL, int G, int NCH>
__device__ __forceinline__ void long_run(const float *__restrict__ carry_, int R,
                                         float *__restrict__ out_, uint32_t row, uint32_t c0,
                                         uint32_t n) {
    const DF_GLOBAL float *__restrict__ carry = gptr(carry_);
    DF_GLOBAL float *__restrict__ out = gptr(out_);
    constexpr int S = kLongBlock / G;
    constexpr int W = CPL * NCH;  // floats per thread
    __shared__ float sh[kLongBlock * W];
    const int slice = threadIdx.x / G, lane = threadIdx.x % G;
    float acc[NCH][CPL];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
#pragma unroll
        for (int q = 0; q < CPL; ++q) acc[c][q] = 0.f;
        const int col = (c * G + lane) * CPL;
        if (col >= R) continue;
        // eight loads in flight, then the adds in the same order as one at
        // a time (k, k + S, k + 2S, ...): the sum is bitwise the same
        uint32_t k = slice;
        for (; k + 7u * S < n; k += 8u * S) {
            float v[8][CPL];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                load_f32<CPL>(carry + (size_t)(c0 + k + u * S) * R + col, v[u]);
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int q = 0; q < CPL; ++q) acc[c][q] += v[u][q];
        }
        for (; k < n; k += S) {
            float v[CPL];
            load_f32<CPL>(carry + (size_t)(c0 + k) * R + col, v);
#pragma unroll
            for (int q = 0; q < CPL; ++q) acc[c][q] += v[q];
        }
    }
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int q = 0; q < CPL; ++q) sh[threadIdx.x * W + c * CPL + q] = acc[c][q];
    __syncthreads();
    for (int half = S / 2; half > 0; half >>= 1) {
        if (slice < half) {
#pragma unroll
            for (int w = 0; w < W; ++w)
                sh[threadIdx.x * W + w] += sh[(threadIdx.x + half * G) * W + w];
        }
        __syncthreads();
    }
    if (slice == 0) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int col = (c * G + lane) * CPL;
            if (col >= R) continue;
            float o[CPL];
            load_f32<CPL>(out + (size_t)row * R + col, o);
#pragma unroll
            for (int q = 0; q < CPL; ++q) o[q] += sh[threadIdx.x * W + c * CPL + q];
            store_vec<CPL>(out + (size_t)row * R + col, o);
        }
    }
}

// Every fix-up of one MTTKRP in one launch (short runs, long runs and empty
// rows own disjoint output rows): blocks [0, nlong) take a long run each, the
// blocks after them the short runs and then the empty rows, one lane group
// each.
template <int CPL, int G, int NCH>
__global__ __launch_bounds__(kLongBlock) void k_fix(
    const uint32_t *__restrict__ runs_long, uint32_t nlong, const uint32_t *__restrict__ runs,
    uint32_t nruns, const float *__restrict__ carry, int R, float *__restrict__ out,
    const uint32_t *__restrict__ empty_rows, uint32_t nempty, uint32_t nempty_groups) {
    if (blockIdx.x < nlong) {
        long_run<CPL, G, NCH>(carry, R, out, runs_long[3 * blockIdx.x],
                              runs_long[3 * blockIdx.x + 1], runs_long[3 * blockIdx.x + 2]);
        return;
    }
    short_runs<CPL, G, NCH>(((blockIdx.x - nlong) * (uint32_t)kLongBlock + threadIdx.x) / G, runs,
                            nruns, carry, R, out, empty_rows, nempty, nempty_groups);
}

// Grouped fix-ups: runs as (tensor, row, c0, n), empty rows as (tensor, row).
template <int CPL, int G, int NCH>
__global__ __launch_bounds__(kBlock) void k_fix_short_group(const GroupMttkrp *__restrict__ desc,
                                                            const uint4 *__restrict__ runs,
                                                            uint32_t nruns,
                                                            const uint2 *__restrict__ empty,
                                                            uint32_t nempty) {
    const uint32_t gid = (blockIdx.x * (uint32_t)kBlock + threadIdx.x) / G;
    const int lane = threadIdx.x % G;
    uint32_t t;
    if (gid < nruns) t = runs[gid].x;
    else if (gid - nruns < nempty) t = empty[gid - nruns].x;
    else return;
    const GroupMttkrp &d = desc[t];
    int col[NCH];
    bool act[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        col[c] = (c * G + lane) * CPL;
        act[c] = col[c] < d.R;
    }
    if (gid < nruns) {
        const uint4 r = runs[gid];
        add_run<CPL, NCH>(d.carry, d.R, d.out, r.y, r.z, r.w, col, act);
    } else {
        zero_row<CPL, NCH>(d.out, d.R, empty[gid - nruns].y, col, act);
    }
}

template <int CPL, int G, int NCH>
__global__ __launch_bounds__(kLongBlock) void k_fix_long_group(const GroupMttkrp *__restrict__ desc,
                                                               const uint4 *__restrict__ runs) {
    const uint4 r = runs[blockIdx.x];
    const GroupMttkrp &d = desc[r.x];
    long_run<CPL, G, NCH>(d.carry, d.R, d.out, r.y, r.z, r.w);
}

// ---- relabeled tables ------------------------------------------------------
// out[r] = in[perm[r]], rows of vr elements of V (a row of R factor entries
// in 16-, 8-, 4- or 2-byte pieces)
template <typename V, bool WIDE>
__global__ __launch_bounds__(256) void k_permute_rows(const V *__restrict__ in,
                                                      const uint32_t *__restrict__ perm,
                                                      int64_t rows, int vr, V *__restrict__ out) {
    const int64_t n = rows * vr;
    for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        int64_t r, c;
        if constexpr (WIDE) {
            r = e / vr;
            c = e - r * vr;
        } else {
            r = (uint32_t)e / (uint32_t)vr;
            c = (uint32_t)e - (uint32_t)r * (uint32_t)vr;
        }
        out[e] = in[(int64_t)perm[r] * vr + c];
    }
}

// out[r * S + c] = in[perm[r] * R + c] for c < R, 0 for R <= c < S (S a
// power of two: the row and column of an element are a shift and a mask)
template <typename T>
__global__ __launch_bounds__(256) void k_permute_pad(const T *__restrict__ in,
                                                     const uint32_t *__restrict__ perm,
                                                     int64_t rows, int R, int log2S,
                                                     T *__restrict__ out) {
    const int64_t n = rows << log2S;
    const int64_t mask = ((int64_t)1 << log2S) - 1;
    for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int64_t r = e >> log2S;
        const int c = (int)(e & mask);
        out[e] = c < R ? in[(int64_t)perm[r] * R + c] : T(0);
    }
}

// out[r * R + c] = in[r * S + c]: a padded MTTKRP result back to R columns
__global__ __launch_bounds__(256) void k_unpad_rows(const float *__restrict__ in, int64_t rows,
                                                    int R, int log2S, float *__restrict__ out) {
    const int64_t n = rows * R;
    for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int64_t r = e / R;
        out[e] = in[(r << log2S) + (e - r * R)];
    }
}

// ---- dispatch --------------------------------------------------------------
template <int V>
using IntC = std::integral_constant<int, V>;
template <typename T>
struct TypeC {
    using type = T;
};

// f(TypeC<T>, IntC<CPL>, IntC<G>, IntC<NCH>) for the kernel shape
template <typename F>
void with_shape(dfacto_dtype dtype, const MttkrpShape &sh, F &&f) {
    auto by_g = [&](auto tc, auto cplc) {
        constexpr int CPL = decltype(cplc)::value;
        if (sh.nch == 1) {
            switch (sh.g) {
                case 2: return f(tc, cplc, IntC<2>{}, IntC<1>{});
                case 4: return f(tc, cplc, IntC<4>{}, IntC<1>{});
                case 8: return f(tc, cplc, IntC<8>{}, IntC<1>{});
                case 16: return f(tc, cplc, IntC<16>{}, IntC<1>{});
                case 32: return f(tc, cplc, IntC<32>{}, IntC<1>{});
                default: return f(tc, cplc, IntC<64>{}, IntC<1>{});
            }
        }
        if constexpr (CPL < 4) {
            if (sh.nch == 2) return f(tc, cplc, IntC<64>{}, IntC<2>{});
        }
        if constexpr (CPL == 1) {
            return f(tc, cplc, IntC<64>{}, IntC<4>{});
        }
        throw Error{DFACTO_E_UNSUPPORTED, "no MTTKRP kernel for this rank"};
    };
    auto by_cpl = [&](auto tc) {
        switch (sh.cpl) {
#if DFACTO_MAX_CPL >= 8
            case 8: return by_g(tc, IntC<8>{});
#endif
            case 4: return by_g(tc, IntC<4>{});
            case 2: return by_g(tc, IntC<2>{});
            default: return by_g(tc, IntC<1>{});
        }
    };
    if (dtype == DFACTO_F32) by_cpl(TypeC<float>{});
    else by_cpl(TypeC<uint16_t>{});
}

// The tables the main kernel gathers from, their row stride (the kernel's
// column count), and for padded tables the padded output rows the kernel
// writes (rows_out of them), copied back to R columns after the fix-ups.
struct Tables {
    const void *leaf = nullptr, *mid = nullptr;
    int stride = 0;
    float *pad_out = nullptr;
    int64_t rows_out = 0;
};

template <typename T, int CPL, int G, int NCH>
// fix/ev: when set, the carry fix-ups go to stream `fix`, ordered after the
// main kernel by `ev` recorded on ctx's stream; carry_in: the carries' buffer
// (else the context's carry workspace)
void run(dfacto_ctx *ctx, const ModeData &md, int R, const Tables &tb, float *out, bool small,
         const void *Froot = nullptr, float *carry_in = nullptr, hipStream_t fix = nullptr,
         hipEvent_t ev = nullptr) {
    hipStream_t s = ctx->stream;
    const uint32_t nchunk = (uint32_t)md.nchunk;
    float *const out_user = out;
    const int R_user = R;
    if (tb.pad_out) {  // the kernels see padded rows of tb.stride columns
        R = tb.stride;
        out = tb.pad_out;
    }
    float *carry = carry_in ? carry_in
                            : (float *)ws_get(ctx, dfacto_ctx::kCarry,
                                              sizeof(float) *
                                                  (size_t)std::max<int64_t>(md.nchunk, 1) * R);
    const T *Fleaf = (const T *)tb.leaf, *Fmid = (const T *)tb.mid;
    constexpr int gpb = kBlock / G;  // groups per block
    if (nchunk > 0) {
        const unsigned blocks = (nchunk + gpb - 1) / gpb;
        if (Froot) {
            if (small)
                hipLaunchKernelGGL((k_mttkrp_res<T, CPL, G, NCH, true>), dim3(blocks),
                                   dim3(kBlock), 0, s, md.stream, md.chunk_start, nchunk, Fleaf,
                                   Fmid, (const T *)Froot, R, out, carry);
            else
                hipLaunchKernelGGL((k_mttkrp_res<T, CPL, G, NCH, false>), dim3(blocks),
                                   dim3(kBlock), 0, s, md.stream, md.chunk_start, nchunk, Fleaf,
                                   Fmid, (const T *)Froot, R, out, carry);
        } else {
            prof_mark(ctx);
            if (small)
                hipLaunchKernelGGL((k_mttkrp<T, CPL, G, NCH, true>), dim3(blocks), dim3(kBlock),
                                   0, s, md.stream, md.chunk_start, nchunk, Fleaf, Fmid, R, out,
                                   carry);
            else
                hipLaunchKernelGGL((k_mttkrp<T, CPL, G, NCH, false>), dim3(blocks), dim3(kBlock),
                                   0, s, md.stream, md.chunk_start, nchunk, Fleaf, Fmid, R, out,
                                   carry);
            prof_mark(ctx);
        }
    }
    if (fix) {
        DF_HIP(hipEventRecord(ev, s));
        DF_HIP(hipStreamWaitEvent(fix, ev, 0));
        s = fix;
    }
    const uint32_t nempty = (uint32_t)md.nempty;
    const uint32_t egroups = nempty == 0 ? 0u : std::min<uint32_t>(nempty, 65536u);
    const uint64_t groups = (uint64_t)md.nruns_short + egroups;
    constexpr int gpl = kLongBlock / G;  // lane groups per fix-up block
    const uint64_t fblocks = (uint64_t)md.nruns_long + (groups + gpl - 1) / gpl;
    if (fblocks > 0)
        hipLaunchKernelGGL((k_fix<CPL, G, NCH>), dim3((unsigned)fblocks), dim3(kLongBlock), 0, s,
                           md.runs_long, (uint32_t)md.nruns_long, md.runs_short,
                           (uint32_t)md.nruns_short, carry, R, out, md.empty_rows, nempty,
                           egroups);
    if (tb.pad_out && tb.rows_out > 0) {
        int log2S = 0;
        while ((1 << log2S) < tb.stride) ++log2S;
        const int64_t n = tb.rows_out * R_user;
        hipLaunchKernelGGL(k_unpad_rows, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 65536)),
                           dim3(256), 0, s, tb.pad_out, tb.rows_out, R_user, log2S, out_user);
    }
    DF_LAUNCHED();
}

}  // namespace

// Row stride of a relabeled mode's gathered copies: rows shorter than a cache
// line (128 bytes) are padded to a power-of-two number of columns, so that no
// row straddles two lines (R = 10 FP32: 40 -> 64 bytes, 13.7 -> 12.3 ms per
// paper-shape launch as measured at R = 16); longer rows keep R.
int table_stride(int R, dfacto_dtype dtype) {
    if ((size_t)R * elem_size(dtype) >= 128) return R;
    int S = 1;
    while (S < R) S <<= 1;
    return S;
}

// Floats per padded output set of a tensor's relabeled modes (0 without
// padding), and the bytes of `sets` of them.
size_t pad_out_stride(const dfacto_tensor *t, int R, dfacto_dtype dtype) {
    const int S = table_stride(R, dtype);
    if (S == R) return 0;
    int64_t rows = 0;
    for (int m = 0; m < 3; ++m)
        if (t->mode[m].perm_leaf) rows = std::max<int64_t>(rows, t->dims[t->mode[m].root]);
    return ((size_t)rows * S + 63) & ~(size_t)63;
}

size_t pad_out_bytes(const dfacto_tensor *t, int R, dfacto_dtype dtype, int sets) {
    return sizeof(float) * pad_out_stride(t, R, dtype) * (size_t)sets;
}

// The column count the main kernel works with for tensor t (the padded
// stride when its relabeled modes pad their rows).
int kernel_cols(const dfacto_tensor *t, int R, dfacto_dtype dtype) {
    return pad_out_stride(t, R, dtype) ? table_stride(R, dtype) : R;
}

namespace {

// Byte offset of the mid table after `rows` leaf rows of `rowb` bytes: a
// whole number of rows that is a multiple of 256 bytes.
size_t mid_offset(int64_t rows, size_t rowb) {
    size_t g = 256, b = rowb;  // gcd(rowb, 256)
    while (b) {
        const size_t r = g % b;
        g = b;
        b = r;
    }
    const size_t m = 256 / g;  // rows per 256-byte multiple
    return ((size_t)rows + m - 1) / m * m * rowb;
}

// rows x R entries of dtype from F into `out` in the order of perm
void launch_permute(dfacto_ctx *ctx, const void *F, const uint32_t *perm, int64_t rows, int R,
                    dfacto_dtype dtype, void *out) {
    if (rows <= 0) return;
    const size_t rowb = (size_t)R * elem_size(dtype);
    auto al = [&](size_t a) {
        return rowb % a == 0 && (uintptr_t)F % a == 0 && (uintptr_t)out % a == 0;
    };
    auto go = [&](auto vt, size_t vb) {
        using V = typename decltype(vt)::type;
        const int vr = (int)(rowb / vb);
        const int64_t n = rows * vr;
        const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
        if (n < ((int64_t)1 << 32))
            hipLaunchKernelGGL((k_permute_rows<V, false>), dim3(grid), dim3(256), 0, ctx->stream,
                               (const V *)F, perm, rows, vr, (V *)out);
        else
            hipLaunchKernelGGL((k_permute_rows<V, true>), dim3(grid), dim3(256), 0, ctx->stream,
                               (const V *)F, perm, rows, vr, (V *)out);
    };
    if (al(16)) go(TypeC<uint4>{}, 16);
    else if (al(8)) go(TypeC<uint2>{}, 8);
    else if (al(4)) go(TypeC<uint32_t>{}, 4);
    else go(TypeC<uint16_t>{}, 2);
    DF_LAUNCHED();
}

// The tables a mode's main kernel gathers from: the factors themselves, or
// for a relabeled mode copies permuted into rank order -- the leaf table,
// then the mid table (mid_offset), in the context's permutation workspace
// or in `buf`.
Tables gather_tables(dfacto_ctx *ctx, const dfacto_tensor *t, int mode, int R, dfacto_dtype dtype,
                     const void *Fleaf, const void *Fmid, void *buf = nullptr, int pad_set = -1) {
    const ModeData &md = t->mode[mode];
    Tables tb;
    tb.stride = R;
    if (!md.perm_leaf) {
        tb.leaf = Fleaf;
        tb.mid = Fmid;
        return tb;
    }
    const int S = pad_set >= 0 ? table_stride(R, dtype) : R;
    if (S != R) {  // rows padded to S (a power of two) columns; see table_stride
        const int64_t dl = t->dims[md.leaf], dm = t->dims[md.mid];
        const size_t es = elem_size(dtype);
        const size_t off_mid = mid_offset(dl, (size_t)S * es);
        char *w = (char *)ws_get(ctx, dfacto_ctx::kPerm, off_mid + (size_t)dm * S * es);
        int log2S = 0;
        while ((1 << log2S) < S) ++log2S;
        auto pad = [&](const void *F, const uint32_t *perm, int64_t rows, void *o) {
            if (rows <= 0) return;
            const unsigned grid =
                (unsigned)std::min<int64_t>((((int64_t)rows << log2S) + 255) / 256, 65536);
            if (dtype == DFACTO_F32)
                hipLaunchKernelGGL(k_permute_pad<float>, dim3(grid), dim3(256), 0, ctx->stream,
                                   (const float *)F, perm, rows, R, log2S, (float *)o);
            else
                hipLaunchKernelGGL(k_permute_pad<uint16_t>, dim3(grid), dim3(256), 0,
                                   ctx->stream, (const uint16_t *)F, perm, rows, R, log2S,
                                   (uint16_t *)o);
            DF_LAUNCHED();
        };
        pad(Fleaf, md.perm_leaf, dl, w);
        pad(Fmid, md.perm_mid, dm, w + off_mid);
        tb.leaf = w;
        tb.mid = w + off_mid;
        tb.stride = S;
        tb.rows_out = t->dims[md.root];
        float *po = (float *)ws_get(ctx, dfacto_ctx::kPadOut, pad_out_bytes(t, R, dtype, pad_set + 1));
        tb.pad_out = po + (size_t)pad_set * pad_out_stride(t, R, dtype);
        return tb;
    }
    const int64_t dl = t->dims[md.leaf], dm = t->dims[md.mid];
    const size_t es = elem_size(dtype);
    const size_t off_mid = mid_offset(dl, (size_t)R * es);
    const size_t total = off_mid + (size_t)dm * R * es;
    char *w = buf ? (char *)buf : (char *)ws_get(ctx, dfacto_ctx::kPerm, total);
    launch_permute(ctx, Fleaf, md.perm_leaf, dl, R, dtype, w);
    launch_permute(ctx, Fmid, md.perm_mid, dm, R, dtype, w + off_mid);
    tb.leaf = w;
    tb.mid = w + off_mid;
    return tb;
}

}  // namespace

void relabeled_tables(const dfacto_tensor *t, int mode, int R, dfacto_dtype dtype, void *buf,
                      const void **leaf, const void **mid) {
    const ModeData &md = t->mode[mode];
    *leaf = buf;
    *mid = (char *)buf + mid_offset(t->dims[md.leaf], (size_t)R * elem_size(dtype));
}

void launch_relabeled_tables(dfacto_ctx *ctx, const dfacto_tensor *t, int mode, int R,
                             dfacto_dtype dtype, const void *Fleaf, const void *Fmid, void *buf) {
    const ModeData &md = t->mode[mode];
    const void *l, *m;
    relabeled_tables(t, mode, R, dtype, buf, &l, &m);
    launch_permute(ctx, Fleaf, md.perm_leaf, t->dims[md.leaf], R, dtype, (void *)l);
    launch_permute(ctx, Fmid, md.perm_mid, t->dims[md.mid], R, dtype, (void *)m);
}

size_t perm_bytes(const dfacto_tensor *t, int R, dfacto_dtype dtype) {
    size_t b = 0;
    // the padded copies of dfacto_mttkrp & co. (the grouped and fixed-array
    // paths keep R columns, fewer bytes)
    const size_t rowb = (size_t)table_stride(R, dtype) * elem_size(dtype);
    for (int m = 0; m < 3; ++m) {
        const ModeData &md = t->mode[m];
        if (!md.perm_leaf) continue;
        b = std::max(b, mid_offset(t->dims[md.leaf], rowb) + (size_t)t->dims[md.mid] * rowb);
    }
    return b;
}

MttkrpShape mttkrp_shape(int R, dfacto_dtype dtype, const void *Fleaf, const void *Fmid,
                         const float *out, bool relabeled) {
    const size_t es = dtype == DFACTO_BF16 ? 2 : 4;
    auto al = [&](size_t a) {
        return ((uintptr_t)Fleaf % a == 0) && ((uintptr_t)Fmid % a == 0) &&
               ((uintptr_t)out % (a * 4 / es) == 0);
    };
    const bool aligned8 = al(8 * es), aligned4 = al(4 * es), aligned2 = al(2 * es);
    int cpl = 1;
    // Eight columns per lane only for BF16 (one 16-byte load per lane): a
    // gather instruction then fetches 16 rows of 64 bytes instead of 8.  For
    // FP32 eight columns are two loads per lane, no fewer instructions.  Only
    // for relabeled gathers (where the most-gathered rows share lines and the
    // wider loads pay: 13.1 -> 12.7 ms per paper-shape launch; with plain
    // gathers they cost 7%: 0.66 -> 0.70 ms at 50M nonzeros), and not below
    // R = 32, where groups of one or two lanes would share each batch of
    // stream entries over too few lanes.
    if (dtype == DFACTO_BF16 && relabeled && R % 8 == 0 && R >= 32 && aligned8 &&
        DFACTO_MAX_CPL >= 8)
        cpl = 8;
    else if (R % 4 == 0 && aligned4 && DFACTO_MAX_CPL >= 4) cpl = 4;
    else if (R % 2 == 0 && aligned2 && DFACTO_MAX_CPL >= 2) cpl = 2;
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

bool mttkrp_small(const dfacto_tensor *t, int mode) {
    // 24-bit row offsets when every index of the leaf, mid and output factor
    // is below 2^24 (then idx * R < 2^32 for R <= 256)
    const ModeData &md = t->mode[mode];
    return t->dims[md.root] < (1 << 24) && t->dims[md.leaf] < (1 << 24) &&
           t->dims[md.mid] < (1 << 24);
}

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
    const bool sm = mttkrp_small(t, mode);
    const Tables tb = gather_tables(ctx, t, mode, R, dtype, Fleaf, Fmid, nullptr, 0);
    const MttkrpShape sh =
        tb.pad_out ? mttkrp_shape(tb.stride, dtype, tb.leaf, tb.mid, tb.pad_out, true)
                   : mttkrp_shape(R, dtype, Fleaf, Fmid, out, md.perm_leaf != nullptr);
    with_shape(dtype, sh, [&](auto tc, auto cplc, auto gc, auto nchc) {
        using T = typename decltype(tc)::type;
        run<T, decltype(cplc)::value, decltype(gc)::value, decltype(nchc)::value>(ctx, md, R, tb,
                                                                                 out, sm);
    });
}

size_t mttkrp_buffers(const dfacto_tensor *t, int mode, int R, dfacto_dtype dtype,
                      size_t *carry_bytes) {
    const ModeData &md = t->mode[mode];
    *carry_bytes = (sizeof(float) * (size_t)std::max<int64_t>(md.nchunk, 1) * R + 255) &
                   ~(size_t)255;
    if (!md.perm_leaf) return 0;
    const size_t rowb = (size_t)R * elem_size(dtype);
    return mid_offset(t->dims[md.leaf], rowb) + (size_t)t->dims[md.mid] * rowb;
}

void launch_mttkrp_in(dfacto_ctx *ctx, const dfacto_tensor *t, int mode, int R,
                      dfacto_dtype dtype, const void *Fleaf, const void *Fmid, float *out,
                      float *carry, void *perm) {
    const ModeData &md = t->mode[mode];
    const MttkrpShape sh = mttkrp_shape(R, dtype, Fleaf, Fmid, out, md.perm_leaf != nullptr);
    const bool sm = mttkrp_small(t, mode);
    const Tables tb = gather_tables(ctx, t, mode, R, dtype, Fleaf, Fmid, perm);
    with_shape(dtype, sh, [&](auto tc, auto cplc, auto gc, auto nchc) {
        using T = typename decltype(tc)::type;
        run<T, decltype(cplc)::value, decltype(gc)::value, decltype(nchc)::value>(ctx, md, R, tb,
                                                                                 out, sm, nullptr,
                                                                                 carry);
    });
}

void launch_mttkrp_split(dfacto_ctx *ctx, const dfacto_tensor *t, int mode, int R,
                         dfacto_dtype dtype, const void *Fleaf, const void *Fmid, float *out,
                         float *carry, hipStream_t fix, hipEvent_t ev) {
    const ModeData &md = t->mode[mode];
    if (ctx->profiling && md.nchunk > 0) {
        const double sf = dtype == DFACTO_BF16 ? 2.0 : 4.0;
        ctx->prof_bytes += 8.0 * (double)t->nnz + 8.0 * (double)md.nfib + 8.0 * (double)md.nroot +
                           4.0 * (double)t->dims[md.root] * R +
                           sf * (double)(t->dims[md.leaf] + t->dims[md.mid]) * R;
        ctx->prof_flops += 2.0 * R * (double)(t->nnz + md.nfib);
    }
    const bool sm = mttkrp_small(t, mode);
    const Tables tb = gather_tables(ctx, t, mode, R, dtype, Fleaf, Fmid, nullptr, mode);
    const MttkrpShape sh =
        tb.pad_out ? mttkrp_shape(tb.stride, dtype, tb.leaf, tb.mid, tb.pad_out, true)
                   : mttkrp_shape(R, dtype, Fleaf, Fmid, out, md.perm_leaf != nullptr);
    with_shape(dtype, sh, [&](auto tc, auto cplc, auto gc, auto nchc) {
        using T = typename decltype(tc)::type;
        run<T, decltype(cplc)::value, decltype(gc)::value, decltype(nchc)::value>(
            ctx, md, R, tb, out, sm, nullptr, carry, fix, ev);
    });
}

void launch_mttkrp_resid(dfacto_ctx *ctx, const dfacto_tensor *t, int mode, int R,
                         dfacto_dtype dtype, const void *Fleaf, const void *Fmid,
                         const void *Froot, float *out) {
    const ModeData &md = t->mode[mode];
    // the root rows share the alignment rule of the gathered rows
    MttkrpShape sh = mttkrp_shape(R, dtype, Fleaf, Fmid, out, false);
    const MttkrpShape sr = mttkrp_shape(R, dtype, Froot, Froot, out, false);
    if (sr.cpl < sh.cpl) sh = sr;
    const bool sm = mttkrp_small(t, mode);
    const Tables tb = gather_tables(ctx, t, mode, R, dtype, Fleaf, Fmid);
    with_shape(dtype, sh, [&](auto tc, auto cplc, auto gc, auto nchc) {
        using T = typename decltype(tc)::type;
        run<T, decltype(cplc)::value, decltype(gc)::value, decltype(nchc)::value>(ctx, md, R, tb,
                                                                                 out, sm, Froot);
    });
}

void launch_gather_probe(dfacto_ctx *ctx, const dfacto_tensor *t, int mode, int R,
                         dfacto_dtype dtype, const void *Fleaf, const void *Fmid, int pattern,
                         float *sink) {
    const ModeData &md = t->mode[mode];
    const MttkrpShape sh = mttkrp_shape(R, dtype, Fleaf, Fmid, sink, md.perm_leaf != nullptr);
    if (sh.nch != 1) throw Error{DFACTO_E_UNSUPPORTED, "the gather probe takes R <= 64 * CPL"};
    if ((pattern == 5 || pattern >= 8) && R > kProbeLdsRowElems)
        throw Error{DFACTO_E_UNSUPPORTED, "the LDS patterns take R <= 64"};
    if (pattern >= 6 && (uint64_t)t->dims[md.leaf] * R * elem_size(dtype) >= 0xFFFFFF00ull)
        throw Error{DFACTO_E_UNSUPPORTED, "the buffer patterns take a leaf table below 4 GB"};
    const bool sm = mttkrp_small(t, mode);
    const uint32_t nchunk = (uint32_t)md.nchunk;
    if (nchunk == 0) return;
    const uint32_t nleaf = (uint32_t)t->dims[md.leaf], nmid = (uint32_t)t->dims[md.mid];
    const Tables tb = gather_tables(ctx, t, mode, R, dtype, Fleaf, Fmid);
    Fleaf = tb.leaf;
    Fmid = tb.mid;
    with_shape(dtype, sh, [&](auto tc, auto cplc, auto gc, auto) {
        using T = typename decltype(tc)::type;
        constexpr int CPL = decltype(cplc)::value, G = decltype(gc)::value;
        if constexpr (G <= 64) {
            const unsigned blocks = (nchunk + kBlock / G - 1) / (kBlock / G);
            auto go = [&](auto kern) {
                prof_mark(ctx);
                hipLaunchKernelGGL(kern, dim3(blocks), dim3(kBlock), 0, ctx->stream, md.stream,
                                   md.chunk_start, nchunk, (const T *)Fleaf, (const T *)Fmid, R,
                                   nleaf, nmid, sink);
                prof_mark(ctx);
            };
            auto by_pat = [&](auto smc) {
                constexpr bool S = decltype(smc)::value;
                switch (pattern) {
                    case 0: return go(k_gather_probe<T, CPL, G, S, 0>);
                    case 1: return go(k_gather_probe<T, CPL, G, S, 1>);
                    case 2: return go(k_gather_probe<T, CPL, G, S, 2>);
                    case 3: return go(k_gather_probe<T, CPL, G, S, 3>);
                    case 4: return go(k_gather_probe<T, CPL, G, S, 4>);
                    case 5: return go(k_gather_probe<T, CPL, G, S, 5>);
                    case 6: return go(k_gather_probe<T, CPL, G, S, 6>);
                    case 7: return go(k_gather_probe<T, CPL, G, S, 7>);
                    case 8: return go(k_gather_probe<T, CPL, G, S, 8>);
                    default: return go(k_gather_probe<T, CPL, G, S, 9>);
                }
            };
            if (sm) by_pat(std::true_type{});
            else by_pat(std::false_type{});
        }
    });
    DF_LAUNCHED();
}

unsigned mttkrp_group_chunks_per_item(const MttkrpShape &sh, unsigned kper) {
    return (unsigned)(kBlock / sh.g) * kper;
}

void launch_mttkrp_group(dfacto_ctx *ctx, dfacto_dtype dtype, const MttkrpShape &sh, bool small,
                         const GroupMttkrp *d_desc, const uint2 *d_items, uint32_t nitems,
                         unsigned grid, unsigned kper) {
    if (nitems == 0) return;
    if (kper < 1 || grid < 1) throw Error{DFACTO_E_INVALID, "grouped MTTKRP launch shape"};
    hipStream_t s = ctx->stream;
    with_shape(dtype, sh, [&](auto tc, auto cplc, auto gc, auto nchc) {
        using T = typename decltype(tc)::type;
        constexpr int CPL = decltype(cplc)::value, G = decltype(gc)::value,
                      NCH = decltype(nchc)::value;
        if (small)
            hipLaunchKernelGGL((k_mttkrp_group<T, CPL, G, NCH, true>), dim3(grid), dim3(kBlock), 0,
                               s, d_desc, d_items, nitems, kper);
        else
            hipLaunchKernelGGL((k_mttkrp_group<T, CPL, G, NCH, false>), dim3(grid), dim3(kBlock),
                               0, s, d_desc, d_items, nitems, kper);
    });
    DF_LAUNCHED();
}

void launch_fix_group(dfacto_ctx *ctx, const MttkrpShape &sh, const GroupMttkrp *d_desc,
                      const uint4 *d_short, uint32_t nshort, const uint2 *d_empty,
                      uint32_t nempty, const uint4 *d_long, uint32_t nlong) {
    hipStream_t s = ctx->stream;
    // the fix-up kernels do not depend on the factor type
    with_shape(DFACTO_F32, sh, [&](auto, auto cplc, auto gc, auto nchc) {
        constexpr int CPL = decltype(cplc)::value, G = decltype(gc)::value,
                      NCH = decltype(nchc)::value;
        const uint64_t groups = (uint64_t)nshort + nempty;
        if (groups > 0) {
            const unsigned blocks = (unsigned)((groups + kBlock / G - 1) / (kBlock / G));
            hipLaunchKernelGGL((k_fix_short_group<CPL, G, NCH>), dim3(blocks), dim3(kBlock), 0, s,
                               d_desc, d_short, nshort, d_empty, nempty);
        }
        if (nlong > 0)
            hipLaunchKernelGGL((k_fix_long_group<CPL, G, NCH>), dim3(nlong), dim3(kLongBlock), 0,
                               s, d_desc, d_long);
    });
    DF_LAUNCHED();
}

}  // namespace dfacto
