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
#define DFACTO_MAX_CPL 4
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
#define MTTKRP_OCCUPANCY __attribute__((amdgpu_waves_per_eu(G <= 32 ? DFACTO_WAVES_PER_EU : 1)))

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

template <>
struct RowLoad<float, 8> {
    static __device__ __forceinline__ void load(const float *p, float (&v)[8]) {
        const float4 x = *reinterpret_cast<const float4 *>(p);
        const float4 y = *reinterpret_cast<const float4 *>(p + 4);
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
};
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
__device__ __forceinline__ void load_f32(const float *p, float (&v)[CPL]) {
    RowLoad<float, CPL>::load(p, v);
}

// ---- main kernel ---------------------------------------------------------
// SMALL: every row index is below 2^24, so row offsets are one 24-bit
// multiply (idx * R < 2^32) instead of 64-bit arithmetic.
// One work chunk (gid) per lane group of G lanes (lane = 0 .. G-1).
// RES: the residual form used by the joint model's ratings term: each
// nonzero's value x becomes x - xhat with xhat = sum_r F_root[root, r]
// F_mid[mid, r] F_leaf[leaf, r] (the CP model at that entry), so the output
// is the MTTKRP of the residual restricted to the stored entries.  The dot
// product is reduced across the group's lanes by xor shuffles (every lane
// ends with the same sum: each step adds two commuted operands).
template <typename T, int CPL, int G, int NCH, bool SMALL, bool RES = false>
__device__ __forceinline__ void mttkrp_chunk(const uint2 *__restrict__ st,
                                             const uint32_t *__restrict__ cstart, uint32_t nchunk,
                                             const T *__restrict__ Fleaf,
                                             const T *__restrict__ Fmid, int R,
                                             float *__restrict__ out, float *__restrict__ carry,
                                             uint32_t gid, int lane,
                                             const T *__restrict__ Froot = nullptr) {
    if (gid >= nchunk) return;
    const uint32_t cs = cstart[gid], ce = cstart[gid + 1];
    if (cs >= ce) return;

    // Per-lane row bases.  Lanes whose columns lie beyond R read column 0
    // instead (in bounds, never stored), so every gather is issued without a
    // branch and the loads of a batch stay in flight together.
    int col[NCH];
    bool act[NCH];
    const T *leafb[NCH], *midb[NCH], *rootb[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        col[c] = (c * G + lane) * CPL;
        act[c] = col[c] < R;
        leafb[c] = Fleaf + (act[c] ? col[c] : 0);
        midb[c] = Fmid + (act[c] ? col[c] : 0);
        rootb[c] = RES ? Froot + (act[c] ? col[c] : 0) : nullptr;
    }
    auto row_off = [&](uint32_t idx) -> size_t {
        if constexpr (SMALL) return (size_t)(uint32_t)__umul24(idx, (uint32_t)R);
        else return (size_t)idx * (size_t)R;
    };

    float acc[NCH][CPL], p[NCH][CPL], mrow[NCH][CPL];
    float rrow[RES ? NCH : 1][CPL];  // the root's factor row (RES only)
    const uint2 h0 = st[cs];
    uint32_t row = h0.y;
    bool cont = !(h0.x & kRootBit);
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
#pragma unroll
        for (int q = 0; q < CPL; ++q) acc[c][q] = p[c][q] = 0.f;
        RowLoad<T, CPL>::load(midb[c] + row_off(h0.x & kIdxMask), mrow[c]);
        if constexpr (RES) RowLoad<T, CPL>::load(rootb[c] + row_off(row), rrow[c]);
    }

    auto flush = [&](uint32_t r_out, bool is_cont) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            if (!act[c]) continue;
            float *dst = is_cont ? carry + (size_t)gid * R + col[c] : out + row_off(r_out) + col[c];
            store_vec<CPL>(dst, acc[c]);
        }
    };

    // Gathers of one batch: every entry's factor row, without branches.
    // Entries at or past the chunk end are still valid stream entries (the
    // next chunk's, or the padding sentinels with index 0), so these loads
    // are in bounds; their values are ignored.
    auto gather = [&](const uint2 (&w)[kUnroll], float (&g)[kUnroll][NCH][CPL]) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const bool hdr = (int32_t)w[u].x < 0;  // kHdrBit is the sign bit
            const size_t off = row_off(w[u].x & kIdxMask);
#pragma unroll
            for (int c = 0; c < NCH; ++c)
                RowLoad<T, CPL>::load((hdr ? midb[c] : leafb[c]) + off, g[u][c]);
        }
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
    mttkrp_chunk<T, CPL, G, NCH, SMALL>(st, cstart, nchunk, Fleaf, Fmid, R, out, carry,
                                        (blockIdx.x * (uint32_t)kBlock + threadIdx.x) / G,
                                        threadIdx.x % G);
}

template <typename T, int CPL, int G, int NCH, bool SMALL>
__global__ __launch_bounds__(kBlock) void k_mttkrp_res(
    const uint2 *__restrict__ st, const uint32_t *__restrict__ cstart, uint32_t nchunk,
    const T *__restrict__ Fleaf, const T *__restrict__ Fmid, const T *__restrict__ Froot, int R,
    float *__restrict__ out, float *__restrict__ carry) {
    mttkrp_chunk<T, CPL, G, NCH, SMALL, true>(st, cstart, nchunk, Fleaf, Fmid, R, out, carry,
                                              (blockIdx.x * (uint32_t)kBlock + threadIdx.x) / G,
                                              threadIdx.x % G, Froot);
}

// Grouped MTTKRP over many tensors of one kernel shape: a persistent grid
// walks the work items (tensor, first chunk of kBlock / G consecutive
// chunks) in a fixed order, item blockIdx.x, blockIdx.x + gridDim.x, ...
template <typename T, int CPL, int G, int NCH, bool SMALL>
__global__ __launch_bounds__(kBlock) MTTKRP_OCCUPANCY void k_mttkrp_group(
    const GroupMttkrp *__restrict__ desc, const uint2 *__restrict__ items, uint32_t nitems) {
    for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const uint2 w = items[it];
        const GroupMttkrp &d = desc[w.x];
        mttkrp_chunk<T, CPL, G, NCH, SMALL>(d.stream, d.chunk_start, d.nchunk,
                                            (const T *)d.Fleaf, (const T *)d.Fmid, d.R, d.out,
                                            d.carry, w.y + threadIdx.x / G, threadIdx.x % G);
    }
}

// ---- fix-up: carries of split rows, and empty rows ------------------------
// out[row] += carry[c0] + ... + carry[c0 + n - 1], in chunk order (one lane
// group; col/act are the lane's column blocks)
template <int CPL, int NCH>
__device__ __forceinline__ void add_run(const float *__restrict__ carry, int R,
                                        float *__restrict__ out, uint32_t row, uint32_t c0,
                                        uint32_t n, const int (&col)[NCH], const bool (&act)[NCH]) {
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
__device__ __forceinline__ void zero_row(float *__restrict__ out, int R, uint32_t row,
                                         const int (&col)[NCH], const bool (&act)[NCH]) {
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
__device__ __forceinline__ void long_run(const float *__restrict__ carry, int R,
                                         float *__restrict__ out, uint32_t row, uint32_t c0,
                                         uint32_t n) {
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

template <typename T, int CPL, int G, int NCH>
// fix/ev: when set, the carry fix-ups go to stream `fix`, ordered after the
// main kernel by `ev` recorded on ctx's stream; carry_in: the carries' buffer
// (else the context's carry workspace)
void run(dfacto_ctx *ctx, const ModeData &md, int R, const void *Fleaf, const void *Fmid,
         float *out, bool small, const void *Froot = nullptr, float *carry_in = nullptr,
         hipStream_t fix = nullptr, hipEvent_t ev = nullptr) {
    hipStream_t s = ctx->stream;
    const uint32_t nchunk = (uint32_t)md.nchunk;
    float *carry = carry_in ? carry_in
                            : (float *)ws_get(ctx, dfacto_ctx::kCarry,
                                              sizeof(float) *
                                                  (size_t)std::max<int64_t>(md.nchunk, 1) * R);
    constexpr int gpb = kBlock / G;  // groups per block
    if (nchunk > 0) {
        const unsigned blocks = (nchunk + gpb - 1) / gpb;
        if (Froot) {
            if (small)
                hipLaunchKernelGGL((k_mttkrp_res<T, CPL, G, NCH, true>), dim3(blocks),
                                   dim3(kBlock), 0, s, md.stream, md.chunk_start, nchunk,
                                   (const T *)Fleaf, (const T *)Fmid, (const T *)Froot, R, out,
                                   carry);
            else
                hipLaunchKernelGGL((k_mttkrp_res<T, CPL, G, NCH, false>), dim3(blocks),
                                   dim3(kBlock), 0, s, md.stream, md.chunk_start, nchunk,
                                   (const T *)Fleaf, (const T *)Fmid, (const T *)Froot, R, out,
                                   carry);
        } else {
            prof_mark(ctx);
            if (small)
                hipLaunchKernelGGL((k_mttkrp<T, CPL, G, NCH, true>), dim3(blocks), dim3(kBlock),
                                   0, s, md.stream, md.chunk_start, nchunk, (const T *)Fleaf,
                                   (const T *)Fmid, R, out, carry);
            else
                hipLaunchKernelGGL((k_mttkrp<T, CPL, G, NCH, false>), dim3(blocks), dim3(kBlock),
                                   0, s, md.stream, md.chunk_start, nchunk, (const T *)Fleaf,
                                   (const T *)Fmid, R, out, carry);
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
    const uint64_t blocks = (uint64_t)md.nruns_long + (groups + gpl - 1) / gpl;
    if (blocks > 0)
        hipLaunchKernelGGL((k_fix<CPL, G, NCH>), dim3((unsigned)blocks), dim3(kLongBlock), 0, s,
                           md.runs_long, (uint32_t)md.nruns_long, md.runs_short,
                           (uint32_t)md.nruns_short, carry, R, out, md.empty_rows, nempty,
                           egroups);
    DF_LAUNCHED();
}

}  // namespace

MttkrpShape mttkrp_shape(int R, dfacto_dtype dtype, const void *Fleaf, const void *Fmid,
                         const float *out) {
    const size_t es = dtype == DFACTO_BF16 ? 2 : 4;
    auto al = [&](size_t a) {
        return ((uintptr_t)Fleaf % a == 0) && ((uintptr_t)Fmid % a == 0) &&
               ((uintptr_t)out % (a * 4 / es) == 0);
    };
    const bool aligned8 = al(8 * es), aligned4 = al(4 * es), aligned2 = al(2 * es);
    int cpl = 1;
    if (R % 8 == 0 && aligned8 && DFACTO_MAX_CPL >= 8) cpl = 8;
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
    const MttkrpShape sh = mttkrp_shape(R, dtype, Fleaf, Fmid, out);
    const bool sm = mttkrp_small(t, mode);
    with_shape(dtype, sh, [&](auto tc, auto cplc, auto gc, auto nchc) {
        using T = typename decltype(tc)::type;
        run<T, decltype(cplc)::value, decltype(gc)::value, decltype(nchc)::value>(
            ctx, md, R, Fleaf, Fmid, out, sm);
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
    const MttkrpShape sh = mttkrp_shape(R, dtype, Fleaf, Fmid, out);
    const bool sm = mttkrp_small(t, mode);
    with_shape(dtype, sh, [&](auto tc, auto cplc, auto gc, auto nchc) {
        using T = typename decltype(tc)::type;
        run<T, decltype(cplc)::value, decltype(gc)::value, decltype(nchc)::value>(
            ctx, md, R, Fleaf, Fmid, out, sm, nullptr, carry, fix, ev);
    });
}

void launch_mttkrp_resid(dfacto_ctx *ctx, const dfacto_tensor *t, int mode, int R,
                         dfacto_dtype dtype, const void *Fleaf, const void *Fmid,
                         const void *Froot, float *out) {
    const ModeData &md = t->mode[mode];
    // the root rows share the alignment rule of the gathered rows
    MttkrpShape sh = mttkrp_shape(R, dtype, Fleaf, Fmid, out);
    const MttkrpShape sr = mttkrp_shape(R, dtype, Froot, Froot, out);
    if (sr.cpl < sh.cpl) sh = sr;
    const bool sm = mttkrp_small(t, mode);
    with_shape(dtype, sh, [&](auto tc, auto cplc, auto gc, auto nchc) {
        using T = typename decltype(tc)::type;
        run<T, decltype(cplc)::value, decltype(gc)::value, decltype(nchc)::value>(
            ctx, md, R, Fleaf, Fmid, out, sm, Froot);
    });
}

unsigned mttkrp_group_chunks_per_item(const MttkrpShape &sh) { return (unsigned)(kBlock / sh.g); }

void launch_mttkrp_group(dfacto_ctx *ctx, dfacto_dtype dtype, const MttkrpShape &sh, bool small,
                         const GroupMttkrp *d_desc, const uint2 *d_items, uint32_t nitems,
                         unsigned grid) {
    if (nitems == 0) return;
    hipStream_t s = ctx->stream;
    with_shape(dtype, sh, [&](auto tc, auto cplc, auto gc, auto nchc) {
        using T = typename decltype(tc)::type;
        constexpr int CPL = decltype(cplc)::value, G = decltype(gc)::value,
                      NCH = decltype(nchc)::value;
        if (small)
            hipLaunchKernelGGL((k_mttkrp_group<T, CPL, G, NCH, true>), dim3(grid), dim3(kBlock), 0,
                               s, d_desc, d_items, nitems);
        else
            hipLaunchKernelGGL((k_mttkrp_group<T, CPL, G, NCH, false>), dim3(grid), dim3(kBlock),
                               0, s, d_desc, d_items, nitems);
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
