// build.hip -- on-device construction of the three fiber-compressed
// flattenings (DFacTo, Section 2.1 eq. (1); Section 3, the CSR storage of
// (X2)^T without zero rows and the precomputed pattern of M^r, Lemmas 3-4).
//
// Pipeline (all on the device, one host readback per size that must be
// known to allocate):
//   validate -> stable LSD radix sort of the coordinates in mode-0 order
//   (i, k, j) -> merge duplicates (sum in input order) -> ||X||^2 ->
//   stable radix sorts by (j, i) and (k, j) for modes 1 and 2 (the mode-0
//   order keeps leaves ascending inside every fiber) -> per mode: fiber
//   and root flags, fiber segments of at most kFiberCap nonzeros, the
//   interleaved header/nonzero stream, empty output rows, work chunks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.hpp"

namespace dfacto {
namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(int64_t n, int per_block = kThreads) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > (1 << 20)) g = 1 << 20;  // grid-stride beyond this
    return (unsigned)g;
}

#define GRID_STRIDE(e, n)                                                           \
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (n);       \
         e += (int64_t)gridDim.x * blockDim.x)

int bits_for(int64_t d) {  // bits needed to store indices 0 .. d-1
    int b = 0;
    while (((int64_t)1 << b) < d) ++b;
    return b;
}

// ---------------------------------------------------------------------------
// simple elementwise kernels
// ---------------------------------------------------------------------------

__global__ void k_validate(const uint32_t *__restrict__ i, const uint32_t *__restrict__ j,
                           const uint32_t *__restrict__ k, const float *__restrict__ v,
                           int64_t n, uint32_t I, uint32_t J, uint32_t K,
                           uint32_t *__restrict__ flag) {
    uint32_t bad = 0;
    GRID_STRIDE(e, n) {
        if (i[e] >= I || j[e] >= J || k[e] >= K) bad |= 1u;
        if (!isfinite(v[e])) bad |= 2u;
    }
    if (bad) atomicOr(flag, bad);
}

__global__ void k_iota(uint32_t *__restrict__ p, int64_t n) {
    GRID_STRIDE(e, n) p[e] = (uint32_t)e;
}

// key = (a << sa) | (b << sb) | c   from coordinate arrays, optionally
// gathered through a permutation.
__global__ void k_make_key(uint64_t *__restrict__ key, const uint32_t *__restrict__ a, int sa,
                           const uint32_t *__restrict__ b, int sb,
                           const uint32_t *__restrict__ c, const uint32_t *__restrict__ perm,
                           int64_t n) {
    GRID_STRIDE(e, n) {
        const int64_t s = perm ? perm[e] : e;
        uint64_t x = 0;
        if (a) x |= (uint64_t)a[s] << sa;
        if (b) x |= (uint64_t)b[s] << sb;
        if (c) x |= (uint64_t)c[s];
        key[e] = x;
    }
}

__global__ void k_gather4(const uint32_t *__restrict__ perm, int64_t n,
                          const uint32_t *__restrict__ a, const uint32_t *__restrict__ b,
                          const uint32_t *__restrict__ c, const float *__restrict__ v,
                          uint32_t *__restrict__ oa, uint32_t *__restrict__ ob,
                          uint32_t *__restrict__ oc, float *__restrict__ ov) {
    GRID_STRIDE(e, n) {
        const uint32_t s = perm[e];
        oa[e] = a[s];
        ob[e] = b[s];
        oc[e] = c[s];
        ov[e] = v[s];
    }
}

// flag[e] = 1 where the sorted coordinate differs from its predecessor
__global__ void k_distinct_flags(const uint32_t *__restrict__ a, const uint32_t *__restrict__ b,
                                 const uint32_t *__restrict__ c, int64_t n,
                                 uint32_t *__restrict__ flag) {
    GRID_STRIDE(e, n) {
        flag[e] = (e == 0 || a[e] != a[e - 1] || b[e] != b[e - 1] || c[e] != c[e - 1]) ? 1u : 0u;
    }
}

// sum each run of equal coordinates in order; write the merged entry
__global__ void k_merge_runs(const uint32_t *__restrict__ flag, const uint32_t *__restrict__ pos,
                             int64_t n, const uint32_t *__restrict__ a,
                             const uint32_t *__restrict__ b, const uint32_t *__restrict__ c,
                             const float *__restrict__ v, uint32_t *__restrict__ oa,
                             uint32_t *__restrict__ ob, uint32_t *__restrict__ oc,
                             float *__restrict__ ov) {
    GRID_STRIDE(e, n) {
        if (!flag[e]) continue;
        float s = v[e];
        for (int64_t t = e + 1; t < n && !flag[t]; ++t) s += v[t];
        const uint32_t o = pos[e];
        if (o >= n) continue;
        oa[o] = a[e];
        ob[o] = b[e];
        oc[o] = c[e];
        ov[o] = s;
    }
}

// per-block partial sums of squares, fixed order
__global__ void k_sumsq_partial(const float *__restrict__ v, int64_t n, double *__restrict__ part) {
    __shared__ double sh[kThreads];
    double s = 0.0;
    GRID_STRIDE(e, n) {
        const double x = v[e];
        s += x * x;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_sum_f64_final(const double *__restrict__ part, int n, double *__restrict__ out) {
    __shared__ double sh[kThreads];
    double s = 0.0;
    for (int e = threadIdx.x; e < n; e += kThreads) s += part[e];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

// ---------------------------------------------------------------------------
// exclusive scan of u32 (three phases, recursive on block sums)
// ---------------------------------------------------------------------------
constexpr int kScanIpt = 8;
constexpr int kScanTile = kThreads * kScanIpt;

__device__ uint32_t block_exclusive_scan(uint32_t x, uint32_t *sh, uint32_t *total) {
    // Hillis-Steele over kThreads values in LDS
    sh[threadIdx.x] = x;
    __syncthreads();
    for (int off = 1; off < kThreads; off <<= 1) {
        uint32_t y = ((int)threadIdx.x >= off) ? sh[threadIdx.x - off] : 0u;
        __syncthreads();
        sh[threadIdx.x] += y;
        __syncthreads();
    }
    const uint32_t incl = sh[threadIdx.x];
    *total = sh[kThreads - 1];
    __syncthreads();
    return incl - x;
}

__global__ void k_scan_reduce(const uint32_t *__restrict__ in, int64_t n,
                              uint32_t *__restrict__ bsum) {
    __shared__ uint32_t sh[kThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint32_t s = 0;
    for (int q = 0; q < kScanIpt; ++q) {
        const int64_t e = base + (int64_t)q * kThreads + threadIdx.x;
        if (e < n) s += in[e];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = sh[0];
}

__global__ void k_scan_apply(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                             int64_t n, const uint32_t *__restrict__ boff) {
    __shared__ uint32_t sh[kThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanIpt;
    uint32_t v[kScanIpt];
    uint32_t s = 0;
    for (int q = 0; q < kScanIpt; ++q) {
        const int64_t e = base + q;
        v[q] = (e < n) ? in[e] : 0u;
        s += v[q];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(s, sh, &total) + (boff ? boff[blockIdx.x] : 0u);
    for (int q = 0; q < kScanIpt; ++q) {
        const int64_t e = base + q;
        if (e < n) out[e] = run;
        run += v[q];
    }
}

// ---------------------------------------------------------------------------
// stable LSD radix sort of (u64 key, u32 value) pairs, 8-bit digits
// ---------------------------------------------------------------------------
constexpr int kRadixIpt = 8;
constexpr int kRadixTile = kThreads * kRadixIpt;

__global__ void k_radix_hist(const uint64_t *__restrict__ keys, int64_t n, int shift,
                             uint32_t *__restrict__ hist, int64_t nblk) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    for (int q = 0; q < kRadixIpt; ++q) {
        const int64_t e = base + (int64_t)q * kThreads + threadIdx.x;
        if (e < n) atomicAdd(&h[(keys[e] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// Keys of a tile are taken in the order q * 256 + tid; a key's rank among
// equal digits of the tile is (keys of earlier slots) + (earlier waves of
// this slot) + (earlier lanes of this wave), the last from 8 ballots that
// isolate the lanes holding the same digit.  The tile's first position for
// digit d is offs[d * nblk + tile] (the exclusive scan of the histograms in
// (digit, tile) order); with kOwn the block forms it itself from the
// histograms (few tiles: nblk reads per thread and a scan over the digits).
constexpr int64_t kRadixOwnMax = 256;  // most tiles for kOwn
template <bool kOwn>
__global__ void k_radix_scatter(const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                                uint64_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                int64_t n, int shift, const uint32_t *__restrict__ offs,
                                int64_t nblk) {
    __shared__ uint32_t s_run[256];
    __shared__ uint32_t s_base[256];
    __shared__ uint32_t s_wc[kThreads / 64][256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    s_run[tid] = 0;
    if constexpr (kOwn) {  // offs holds the histograms here
        const uint32_t *hd = offs + (int64_t)tid * nblk;
        uint32_t tot = 0, pre = 0;
        for (int64_t b = 0; b < nblk; ++b) {
            const uint32_t c = hd[b];
            tot += c;
            pre += (b < (int64_t)blockIdx.x) ? c : 0u;
        }
        // inclusive scan of the digit totals (s_base as scratch), then
        // exclusive = inclusive - own total
        s_base[tid] = tot;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            const uint32_t v = tid >= o ? s_base[tid - o] : 0u;
            __syncthreads();
            s_base[tid] += v;
            __syncthreads();
        }
        s_base[tid] = s_base[tid] - tot + pre;
    } else {
        s_base[tid] = offs[(int64_t)tid * nblk + blockIdx.x];
    }
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    for (int q = 0; q < kRadixIpt; ++q) {
        const int64_t e = base + (int64_t)q * kThreads + tid;
        const bool valid = e < n;
        const uint64_t key = valid ? kin[e] : 0ull;
        const uint32_t val = valid ? vin[e] : 0u;
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) s_wc[w][tid] = 0;
        __syncthreads();
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bal = __ballot(bit);
            m &= bit ? bal : ~bal;
        }
        const uint32_t rank = (uint32_t)__popcll(m & lt);
        if (valid && rank == 0) s_wc[wave][d] = (uint32_t)__popcll(m);
        __syncthreads();
        if (valid) {
            uint32_t pre = s_run[d];
            for (int w = 0; w < wave; ++w) pre += s_wc[w][d];
            const uint32_t pos = s_base[d] + pre + rank;
            if ((int64_t)pos < n) {  // always true for consistent histograms
                kout[pos] = key;
                vout[pos] = val;
            }
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) add += s_wc[w][tid];
        s_run[tid] += add;
    }
}

// ---------------------------------------------------------------------------
// per-mode stream construction
// ---------------------------------------------------------------------------

__global__ void k_fiber_flags(const uint32_t *__restrict__ root, const uint32_t *__restrict__ mid,
                              int64_t n, uint32_t *__restrict__ fs, uint32_t *__restrict__ rs) {
    GRID_STRIDE(e, n) {
        const bool r = (e == 0) || root[e] != root[e - 1];
        const bool f = r || mid[e] != mid[e - 1];
        fs[e] = f ? 1u : 0u;
        rs[e] = r ? 1u : 0u;
    }
}

__global__ void k_fiber_start_pos(const uint32_t *__restrict__ fs, const uint32_t *__restrict__ fid,
                                  int64_t n, int64_t nfib, uint32_t *__restrict__ fptr) {
    GRID_STRIDE(e, n) {
        if (fs[e] && fid[e] < nfib) fptr[fid[e]] = (uint32_t)e;
    }
}

// h[e] = 1 if a header precedes nonzero e: at every fiber start and every
// kFiberCap nonzeros inside a fiber.
__global__ void k_header_flags(const uint32_t *__restrict__ fs, const uint32_t *__restrict__ fid,
                               const uint32_t *__restrict__ fptr, int64_t n, int64_t nfib,
                               uint32_t *__restrict__ h) {
    GRID_STRIDE(e, n) {
        const uint32_t f = fid[e] + fs[e] - 1u;  // fiber index (inclusive count - 1)
        const uint32_t off = (f < nfib) ? (uint32_t)e - fptr[f] : 0u;
        h[e] = (fs[e] || (off % (uint32_t)kFiberCap) == 0u) ? 1u : 0u;
    }
}

// inv_leaf / inv_mid (or null): the relabeled index of each leaf / mid row
__global__ void k_emit_stream(const uint32_t *__restrict__ root, const uint32_t *__restrict__ mid,
                              const uint32_t *__restrict__ leaf, const float *__restrict__ val,
                              const uint32_t *__restrict__ h, const uint32_t *__restrict__ hex,
                              const uint32_t *__restrict__ rs, int64_t n, int64_t L,
                              const uint32_t *__restrict__ inv_leaf,
                              const uint32_t *__restrict__ inv_mid, uint2 *__restrict__ st) {
    GRID_STRIDE(e, n) {
        const uint32_t pos = (uint32_t)e + hex[e] + h[e];
        if ((int64_t)pos >= L) continue;  // never taken when the scan is consistent
        if (h[e]) {
            const uint32_t m = inv_mid ? inv_mid[mid[e]] : mid[e];
            st[pos - 1] = make_uint2(kHdrBit | (rs[e] ? kRootBit : 0u) | m, root[e]);
        }
        st[pos] = make_uint2(inv_leaf ? inv_leaf[leaf[e]] : leaf[e], __float_as_uint(val[e]));
    }
}

// Gathers per row: every nonzero gathers its leaf row, every header (fiber
// start or segment start) its mid row.  Skewed indices put millions of
// counts on a few rows, so the counts are not accumulated with atomics (they
// serialize on those rows' addresses): the gathered indices are radix-sorted
// and each row's count is the length of its run.
// (k_count_input) the indices to sort: all of them, or those with flag[e]
// set, compacted through pos (the exclusive scan of flag)
__global__ void k_count_input(const uint32_t *__restrict__ idx, const uint32_t *__restrict__ flag,
                              const uint32_t *__restrict__ pos, int64_t n,
                              uint64_t *__restrict__ key, uint32_t *__restrict__ val) {
    GRID_STRIDE(e, n) {
        if (!flag) {
            key[e] = idx[e];
            val[e] = 0u;
        } else if (flag[e]) {
            key[pos[e]] = idx[e];
            val[pos[e]] = 0u;
        }
    }
}

// [beg[r], end[r]) = the run of row r in the sorted keys (rows absent from
// the keys keep the zeros they were filled with)
__global__ void k_run_bounds(const uint64_t *__restrict__ key, int64_t n,
                             uint32_t *__restrict__ beg, uint32_t *__restrict__ end) {
    GRID_STRIDE(e, n) {
        const uint64_t k = key[e];
        if (e == 0 || key[e - 1] != k) beg[k] = (uint32_t)e;
        if (e == n - 1 || key[e + 1] != k) end[k] = (uint32_t)(e + 1);
    }
}

__global__ void k_run_lengths(const uint32_t *__restrict__ beg, const uint32_t *__restrict__ end,
                              int64_t rows, uint32_t *__restrict__ cnt) {
    GRID_STRIDE(r, rows) cnt[r] = end[r] - beg[r];
}

// sort key: count descending (a stable sort keeps equal counts in index order)
__global__ void k_count_keys(const uint32_t *__restrict__ cnt, int64_t n,
                             uint64_t *__restrict__ key, uint32_t *__restrict__ idx) {
    GRID_STRIDE(e, n) {
        key[e] = (uint64_t)(0xFFFFFFFFu - cnt[e]);
        idx[e] = (uint32_t)e;
    }
}

__global__ void k_invert(const uint32_t *__restrict__ perm, int64_t n, uint32_t *__restrict__ inv) {
    GRID_STRIDE(e, n) inv[perm[e]] = (uint32_t)e;
}

__global__ void k_fill_pad(uint2 *__restrict__ st, int64_t from, int64_t count) {
    GRID_STRIDE(e, count) st[from + e] = make_uint2(kHdrBit | kRootBit, 0u);
}

__global__ void k_mark_rows(const uint32_t *__restrict__ root, const uint32_t *__restrict__ rs,
                            int64_t n, int64_t nrows, uint32_t *__restrict__ mark) {
    GRID_STRIDE(e, n) {
        if (rs[e] && root[e] < nrows) mark[root[e]] = 0u;
    }
}

__global__ void k_fill_u32(uint32_t *__restrict__ p, int64_t n, uint32_t v) {
    GRID_STRIDE(e, n) p[e] = v;
}

__global__ void k_compact_rows(const uint32_t *__restrict__ mark, const uint32_t *__restrict__ pos,
                               int64_t n, uint32_t *__restrict__ out) {
    GRID_STRIDE(e, n) {
        if (mark[e]) out[pos[e]] = (uint32_t)e;
    }
}

// chunk c starts at the first header at or after c * len (or at the end)
__global__ void k_chunk_starts(const uint2 *__restrict__ st, int64_t nentry, int64_t nchunk,
                               int len, uint32_t *__restrict__ cs) {
    GRID_STRIDE(c, nchunk + 1) {
        int64_t p = c * (int64_t)len;
        if (c == nchunk || p >= nentry) {
            p = nentry;
        } else {
            while (p < nentry && !(st[p].x & kHdrBit)) ++p;
        }
        cs[c] = (uint32_t)p;
    }
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------

// Transient build buffers, stream-ordered (from the context's memory
// source, freed on the build stream), so building one tensor never waits for
// unrelated work on the device.
struct Scratch {
    hipStream_t s;
    DevMem mem;
    std::vector<void *> ptrs;
    Scratch(hipStream_t st, const DevMem &m) : s(st), mem(m) {}
    ~Scratch() {
        for (void *p : ptrs) mem.free(p, s);
    }
    template <typename T>
    T *alloc(int64_t n) {
        void *p = nullptr;
        const size_t bytes = sizeof(T) * (size_t)std::max<int64_t>(n, 1);
        if (mem.arena && (p = mem.arena->take(bytes))) return (T *)p;  // freed with the arena
        if (mem.alloc(&p, bytes, s) != hipSuccess) {
            (void)hipGetLastError();
            throw Error{DFACTO_E_NOMEM, "device allocation of " + std::to_string(bytes) +
                                            " bytes failed while building the flattenings"};
        }
        ptrs.push_back(p);
        return (T *)p;
    }
    void release(void *p) {
        for (auto &q : ptrs)
            if (q == p) {
                mem.free(q, s);
                q = nullptr;
            }
    }
};

// Tensor memory.  Arrays up to kSlabTake bytes (chunk starts, run lists,
// empty rows, the streams of small tensors) share slabs of kSlabBytes, so a
// small tensor makes a few allocations instead of about fifteen.
constexpr size_t kSlabTake = (size_t)256 << 10, kSlabBytes = (size_t)1 << 20;

void *tensor_alloc_bytes(dfacto_tensor *t, size_t bytes) {
    bytes = (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
    auto raw = [&](size_t b) {
        void *p = nullptr;
        const hipError_t e =
            t->alloc_stream ? t->mem.alloc(&p, b, t->alloc_stream) : hipMalloc(&p, b);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw Error{DFACTO_E_NOMEM, "device allocation of " + std::to_string(b) +
                                            " bytes failed for the flattenings"};
        }
        t->allocations.push_back(p);
        t->bytes += b;
        return (char *)p;
    };
    if (bytes > kSlabTake) return raw(bytes);
    if (bytes > t->slab_left) {
        t->slab = raw(kSlabBytes);
        t->slab_left = kSlabBytes;
    }
    void *p = t->slab;
    t->slab += bytes;
    t->slab_left -= bytes;
    return p;
}

template <typename T>
T *tensor_alloc(dfacto_tensor *t, int64_t n) {
    return (T *)tensor_alloc_bytes(t, sizeof(T) * (size_t)std::max<int64_t>(n, 1));
}

// out[q] = *a[q] + *b[q] for several scan totals (last offset plus last
// flag of an exclusive scan), one wait
template <int N>
void read_back_sums(const uint32_t *const (&a)[N], const uint32_t *const (&b)[N], int64_t (&out)[N],
                    hipStream_t s) {
    uint32_t h[2 * N];
    for (int q = 0; q < N; ++q) {
        DF_HIP(hipMemcpyAsync(&h[2 * q], a[q], sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        DF_HIP(hipMemcpyAsync(&h[2 * q + 1], b[q], sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    }
    DF_HIP(hipStreamSynchronize(s));
    for (int q = 0; q < N; ++q) out[q] = (int64_t)h[2 * q] + h[2 * q + 1];
}

void radix_sort(uint64_t *&keys, uint32_t *&vals, uint64_t *&kalt, uint32_t *&valt, int64_t n,
                int bits, Scratch &sc, hipStream_t s) {
    if (n <= 1 || bits <= 0) return;
    const int64_t nblk = (n + kRadixTile - 1) / kRadixTile;
    uint32_t *hist = sc.alloc<uint32_t>(256 * nblk);
    uint32_t *offs = sc.alloc<uint32_t>(256 * nblk);
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nblk), dim3(kThreads), 0, s, keys, n,
                           shift, hist, nblk);
        if (nblk <= kRadixOwnMax) {  // two launches per pass instead of five
            hipLaunchKernelGGL(k_radix_scatter<true>, dim3((unsigned)nblk), dim3(kThreads), 0, s,
                               keys, vals, kalt, valt, n, shift, hist, nblk);
        } else {
            scan_exclusive_u32(hist, offs, 256 * nblk, s, &sc.mem);
            hipLaunchKernelGGL(k_radix_scatter<false>, dim3((unsigned)nblk), dim3(kThreads), 0, s,
                               keys, vals, kalt, valt, n, shift, offs, nblk);
        }
        std::swap(keys, kalt);
        std::swap(vals, valt);
    }
    DF_LAUNCHED();
    sc.release(hist);
    sc.release(offs);
}

__global__ void k_chunk_heads(const uint2 *__restrict__ st, const uint32_t *__restrict__ cs,
                              int64_t nchunk, uint2 *__restrict__ heads) {
    GRID_STRIDE(c, nchunk) {
        const uint32_t a = cs[c];
        heads[c] = (a < cs[c + 1]) ? st[a] : make_uint2(kHdrBit | kRootBit, 0u);
    }
}

// Rows split across chunks: a maximal sequence of chunks whose first header
// continues the same row (no ROOT bit) forms one run of carries.
// The heads of the mode's chunks, copied to `heads` (complete at the build's
// next wait); finish_runs forms the run lists from them.
void chunk_heads(ModeData &md, hipStream_t s, Scratch &sc, std::vector<uint2> &heads) {
    heads.assign((size_t)md.nchunk, make_uint2(0u, 0u));
    if (md.nchunk == 0) return;
    uint2 *dh = sc.alloc<uint2>(md.nchunk);
    hipLaunchKernelGGL(k_chunk_heads, dim3(grid_for(md.nchunk)), dim3(kThreads), 0, s, md.stream,
                       md.chunk_start, md.nchunk, dh);
    DF_LAUNCHED();
    DF_HIP(hipMemcpyAsync(heads.data(), dh, sizeof(uint2) * md.nchunk, hipMemcpyDeviceToHost, s));
}

void finish_runs(dfacto_tensor *t, ModeData &md, hipStream_t s, const std::vector<uint2> &heads) {
    if (md.nchunk == 0) return;
    std::vector<uint32_t> shortr, longr;
    int64_t c = 0;
    while (c < md.nchunk) {
        if (heads[c].x & kRootBit) {
            ++c;
            continue;
        }
        const uint32_t row = heads[c].y;
        int64_t e = c + 1;
        while (e < md.nchunk && !(heads[e].x & kRootBit) && heads[e].y == row) ++e;
        auto &dst = (e - c <= kShortRun) ? shortr : longr;
        dst.push_back(row);
        dst.push_back((uint32_t)c);
        dst.push_back((uint32_t)(e - c));
        c = e;
    }
    md.nruns_short = (int64_t)shortr.size() / 3;
    md.nruns_long = (int64_t)longr.size() / 3;
    md.runs_short = tensor_alloc<uint32_t>(t, (int64_t)shortr.size());
    md.runs_long = tensor_alloc<uint32_t>(t, (int64_t)longr.size());
    if (!shortr.empty())
        DF_HIP(hipMemcpyAsync(md.runs_short, shortr.data(), sizeof(uint32_t) * shortr.size(),
                              hipMemcpyHostToDevice, s));
    if (!longr.empty())
        DF_HIP(hipMemcpyAsync(md.runs_long, longr.data(), sizeof(uint32_t) * longr.size(),
                              hipMemcpyHostToDevice, s));
    // the host lists move into the mode data (same buffers), so they outlive
    // the asynchronous copies; the build waits for its stream at the end
    md.runs_short_host = std::move(shortr);
    md.runs_long_host = std::move(longr);
}

// cnt[r] = occurrences of row r among the n indices idx (flag null) or among
// those with flag[e] set (m of them; pos = the exclusive scan of flag), for
// rows r < rows.
void count_rows(const uint32_t *idx, const uint32_t *flag, const uint32_t *pos, int64_t n,
                int64_t m, int64_t rows, uint32_t *cnt, Scratch &sc, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(rows)), dim3(kThreads), 0, s, cnt, rows, 0u);
    DF_LAUNCHED();
    if (m == 0) return;
    uint64_t *key = sc.alloc<uint64_t>(m), *kalt = sc.alloc<uint64_t>(m);
    uint32_t *val = sc.alloc<uint32_t>(m), *valt = sc.alloc<uint32_t>(m);
    hipLaunchKernelGGL(k_count_input, dim3(grid_for(n)), dim3(kThreads), 0, s, idx, flag, pos, n,
                       key, val);
    DF_LAUNCHED();
    radix_sort(key, val, kalt, valt, m, bits_for(rows), sc, s);
    uint32_t *beg = sc.alloc<uint32_t>(rows), *end = sc.alloc<uint32_t>(rows);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(rows)), dim3(kThreads), 0, s, beg, rows, 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(rows)), dim3(kThreads), 0, s, end, rows, 0u);
    hipLaunchKernelGGL(k_run_bounds, dim3(grid_for(m)), dim3(kThreads), 0, s, key, m, beg, end);
    hipLaunchKernelGGL(k_run_lengths, dim3(grid_for(rows)), dim3(kThreads), 0, s, beg, end, rows,
                       cnt);
    DF_LAUNCHED();
    sc.release(end);
    sc.release(beg);
    sc.release(valt);
    sc.release(val);
    sc.release(kalt);
    sc.release(key);
}

// The order of a gathered table's rows by decreasing gather count (ties by
// index): perm[r] = the row ranked r (tensor memory).
uint32_t *relabel_order(dfacto_tensor *t, const uint32_t *cnt, int64_t rows, Scratch &sc,
                        hipStream_t s) {
    uint64_t *key = sc.alloc<uint64_t>(rows), *kalt = sc.alloc<uint64_t>(rows);
    uint32_t *idx = sc.alloc<uint32_t>(rows), *ialt = sc.alloc<uint32_t>(rows);
    hipLaunchKernelGGL(k_count_keys, dim3(grid_for(rows)), dim3(kThreads), 0, s, cnt, rows, key,
                       idx);
    DF_LAUNCHED();
    radix_sort(key, idx, kalt, ialt, rows, 32, sc, s);
    uint32_t *perm = tensor_alloc<uint32_t>(t, rows);
    DF_HIP(hipMemcpyAsync(perm, idx, sizeof(uint32_t) * (size_t)rows, hipMemcpyDeviceToDevice, s));
    return perm;
}

// Mode m's flattening from its nonzeros in (root, mid) order; the chunk
// heads for its run lists land in `heads` at the build's next wait.
void build_mode(dfacto_ctx *ctx, dfacto_tensor *t, int m, const uint32_t *root,
                const uint32_t *mid, const uint32_t *leaf, const float *val, int64_t n,
                std::vector<uint2> &heads) {
    hipStream_t s = ctx->stream;
    ModeData &md = t->mode[m];
    const int64_t nrows = t->dims[md.root];
    Scratch sc(s, ctx->mem);
    const int chunk_len = t->chunk_len;
    md.chunk_len = chunk_len;
    if (n == 0) {
        md.nentry = 0;
        md.nfib = md.nroot = 0;
        md.stream = tensor_alloc<uint2>(t, kStreamPad);
        hipLaunchKernelGGL(k_fill_pad, dim3(1), dim3(kThreads), 0, s, md.stream, (int64_t)0,
                           (int64_t)kStreamPad);
        md.nchunk = 0;
        md.chunk_start = tensor_alloc<uint32_t>(t, 1);
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kThreads), 0, s, md.chunk_start,
                           (int64_t)1, 0u);
        md.nempty = nrows;
        md.empty_rows = tensor_alloc<uint32_t>(t, nrows);
        uint32_t *mark = sc.alloc<uint32_t>(nrows);
        hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(nrows)), dim3(kThreads), 0, s, mark, nrows,
                           1u);
        uint32_t *pos = sc.alloc<uint32_t>(nrows);
        scan_exclusive_u32(mark, pos, nrows, s, &sc.mem);
        hipLaunchKernelGGL(k_compact_rows, dim3(grid_for(nrows)), dim3(kThreads), 0, s, mark, pos,
                           nrows, md.empty_rows);
        DF_LAUNCHED();
        DF_HIP(hipStreamSynchronize(s));
        return;
    }
    uint32_t *fs = sc.alloc<uint32_t>(n);
    uint32_t *rs = sc.alloc<uint32_t>(n);
    uint32_t *fid = sc.alloc<uint32_t>(n);
    hipLaunchKernelGGL(k_fiber_flags, dim3(grid_for(n)), dim3(kThreads), 0, s, root, mid, n, fs,
                       rs);
    scan_exclusive_u32(fs, fid, n, s, &sc.mem);
    // fiber starts (n bounds the fiber count: no wait for it here)
    uint32_t *fptr = sc.alloc<uint32_t>(n);
    hipLaunchKernelGGL(k_fiber_start_pos, dim3(grid_for(n)), dim3(kThreads), 0, s, fs, fid, n, n,
                       fptr);
    uint32_t *h = sc.alloc<uint32_t>(n);
    hipLaunchKernelGGL(k_header_flags, dim3(grid_for(n)), dim3(kThreads), 0, s, fs, fid, fptr, n,
                       n, h);
    sc.release(fptr);
    uint32_t *hex = sc.alloc<uint32_t>(n);
    scan_exclusive_u32(h, hex, n, s, &sc.mem);
    // roots and empty output rows
    uint32_t *mark = sc.alloc<uint32_t>(nrows);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(nrows)), dim3(kThreads), 0, s, mark, nrows, 1u);
    hipLaunchKernelGGL(k_mark_rows, dim3(grid_for(n)), dim3(kThreads), 0, s, root, rs, n, nrows,
                       mark);
    uint32_t *rpos = sc.alloc<uint32_t>(nrows);
    scan_exclusive_u32(mark, rpos, nrows, s, &sc.mem);
    DF_LAUNCHED();
    // fibers, headers and empty rows, one wait
    int64_t cnt[3];
    read_back_sums<3>({fid + n - 1, hex + n - 1, rpos + nrows - 1},
                      {fs + n - 1, h + n - 1, mark + nrows - 1}, cnt, s);
    md.nfib = cnt[0];
    const int64_t nhdr = cnt[1];
    md.nempty = cnt[2];
    const int64_t L = n + nhdr;
    if (L > (int64_t)0xFFFFFFFFu - (1 << 20))
        throw Error{DFACTO_E_UNSUPPORTED, "nonzeros plus fiber headers exceed 2^32 - 2^20"};
    md.nentry = L;
    // relabeled gathers: ranks by decreasing gather count per gathered table
    const uint32_t *inv_leaf = nullptr, *inv_mid = nullptr;
    if (t->relabel) {
        const int64_t dl = t->dims[md.leaf], dm = t->dims[md.mid];
        uint32_t *cl = sc.alloc<uint32_t>(dl), *cm = sc.alloc<uint32_t>(dm);
        count_rows(leaf, nullptr, nullptr, n, n, dl, cl, sc, s);
        count_rows(mid, h, hex, n, nhdr, dm, cm, sc, s);
        md.perm_leaf = relabel_order(t, cl, dl, sc, s);
        md.perm_mid = relabel_order(t, cm, dm, sc, s);
        uint32_t *il = sc.alloc<uint32_t>(dl), *im = sc.alloc<uint32_t>(dm);
        hipLaunchKernelGGL(k_invert, dim3(grid_for(dl)), dim3(kThreads), 0, s, md.perm_leaf, dl, il);
        hipLaunchKernelGGL(k_invert, dim3(grid_for(dm)), dim3(kThreads), 0, s, md.perm_mid, dm, im);
        DF_LAUNCHED();
        inv_leaf = il;
        inv_mid = im;
    }
    md.stream = tensor_alloc<uint2>(t, L + kStreamPad);
    hipLaunchKernelGGL(k_emit_stream, dim3(grid_for(n)), dim3(kThreads), 0, s, root, mid, leaf, val,
                       h, hex, rs, n, L, inv_leaf, inv_mid, md.stream);
    hipLaunchKernelGGL(k_fill_pad, dim3(1), dim3(kThreads), 0, s, md.stream, L,
                       (int64_t)kStreamPad);
    md.nroot = nrows - md.nempty;
    md.empty_rows = tensor_alloc<uint32_t>(t, md.nempty);
    hipLaunchKernelGGL(k_compact_rows, dim3(grid_for(nrows)), dim3(kThreads), 0, s, mark, rpos,
                       nrows, md.empty_rows);
    // work chunks
    md.nchunk = (L + chunk_len - 1) / chunk_len;
    md.chunk_start = tensor_alloc<uint32_t>(t, md.nchunk + 1);
    hipLaunchKernelGGL(k_chunk_starts, dim3(grid_for(md.nchunk + 1)), dim3(kThreads), 0, s,
                       md.stream, L, md.nchunk, chunk_len, md.chunk_start);
    DF_LAUNCHED();
    chunk_heads(md, s, sc, heads);
}

// 1 where a stream entry opens an output row (a ROOT header)
__global__ void k_root_flags(const uint2 *__restrict__ st, int64_t n, uint32_t *__restrict__ f) {
    GRID_STRIDE(e, n) f[e] = ((st[e].x & (kHdrBit | kRootBit)) == (kHdrBit | kRootBit)) ? 1u : 0u;
}

// the q-th row opening of the stream at pos[q] covers [pos[q], pos[q+1])
__global__ void k_row_ranges(const uint2 *__restrict__ st, const uint32_t *__restrict__ flag,
                             const uint32_t *__restrict__ off, int64_t n, uint32_t *__restrict__ pos) {
    GRID_STRIDE(e, n) if (flag[e]) pos[off[e]] = (uint32_t)e;
}

__global__ void k_store_ranges(const uint2 *__restrict__ st, const uint32_t *__restrict__ pos,
                               int64_t nroot, int64_t n, uint2 *__restrict__ range) {
    GRID_STRIDE(q, nroot) {
        const uint32_t b = pos[q];
        const uint32_t e = (q + 1 < nroot) ? pos[q + 1] : (uint32_t)n;
        range[st[b].y] = make_uint2(b, e);
    }
}

}  // namespace

void scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t n, hipStream_t s,
                        const DevMem *mem) {
    if (n <= 0) return;
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(kThreads), 0, s, in, out, n,
                           (const uint32_t *)nullptr);
        return;
    }
    Scratch sc(s, mem ? *mem : DevMem{});
    uint32_t *bsum = sc.alloc<uint32_t>(nb), *boff = sc.alloc<uint32_t>(nb);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kThreads), 0, s, in, n, bsum);
    scan_exclusive_u32(bsum, boff, nb, s, &sc.mem);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kThreads), 0, s, in, out, n,
                       (const uint32_t *)boff);
}

void build_row_ranges(dfacto_ctx *ctx, dfacto_tensor *t) {
    hipStream_t s = ctx->stream;
    Scratch sc(s, ctx->mem);
    for (int m = 0; m < 2; ++m) {
        const ModeData &md = t->mode[m];
        const int64_t rows = t->dims[md.root], n = md.nentry;
        uint2 *range = tensor_alloc<uint2>(t, rows);
        DF_HIP(hipMemsetAsync(range, 0, sizeof(uint2) * (size_t)rows, s));
        if (n > 0 && md.nroot > 0) {
            uint32_t *flag = sc.alloc<uint32_t>(n), *off = sc.alloc<uint32_t>(n);
            uint32_t *pos = sc.alloc<uint32_t>(md.nroot);
            hipLaunchKernelGGL(k_root_flags, dim3(grid_for(n)), dim3(kThreads), 0, s, md.stream, n,
                               flag);
            scan_exclusive_u32(flag, off, n, s, &sc.mem);
            hipLaunchKernelGGL(k_row_ranges, dim3(grid_for(n)), dim3(kThreads), 0, s, md.stream,
                               flag, off, n, pos);
            hipLaunchKernelGGL(k_store_ranges, dim3(grid_for(md.nroot)), dim3(kThreads), 0, s,
                               md.stream, pos, md.nroot, n, range);
            DF_LAUNCHED();
        }
        t->row_range[m] = range;
    }
    // rows longer than kJointSeg entries become segments of kJointSeg
    std::vector<uint2> hr, seg[2];
    std::vector<uint4> heavy[2];
    for (int m = 0; m < 2; ++m) {
        const int64_t rows = t->dims[t->mode[m].root];
        hr.resize((size_t)rows);
        DF_HIP(hipMemcpyAsync(hr.data(), t->row_range[m], sizeof(uint2) * (size_t)rows,
                              hipMemcpyDeviceToHost, s));
        DF_HIP(hipStreamSynchronize(s));
        for (int64_t r = 0; r < rows; ++r) {
            const uint32_t b = hr[r].x, e = hr[r].y;
            if (e - b <= (uint32_t)kJointSeg) continue;
            heavy[m].push_back(make_uint4((uint32_t)r, (uint32_t)seg[m].size(),
                                          (e - b + kJointSeg - 1) / kJointSeg, 0u));
            for (uint32_t x = b; x < e; x += kJointSeg)
                seg[m].push_back(make_uint2(x, std::min<uint32_t>(e, x + kJointSeg)));
        }
        t->nseg[m] = (int64_t)seg[m].size();
        t->nheavy[m] = (int64_t)heavy[m].size();
        t->seg_range[m] = tensor_alloc<uint2>(t, t->nseg[m]);
        t->heavy[m] = tensor_alloc<uint4>(t, t->nheavy[m]);
        if (t->nseg[m] > 0) {
            DF_HIP(hipMemcpyAsync(t->seg_range[m], seg[m].data(), sizeof(uint2) * seg[m].size(),
                                  hipMemcpyHostToDevice, s));
            DF_HIP(hipMemcpyAsync(t->heavy[m], heavy[m].data(), sizeof(uint4) * heavy[m].size(),
                                  hipMemcpyHostToDevice, s));
        }
    }
    DF_HIP(hipStreamSynchronize(s));
}

void build_tensor(dfacto_ctx *ctx, dfacto_tensor *t, const uint32_t *d_i, const uint32_t *d_j,
                  const uint32_t *d_k, const float *d_val) {
    hipStream_t s = ctx->stream;
    const int64_t n = t->nnz;
    Scratch sc(s, ctx->mem);
    static const int ROOT[3] = {0, 1, 2}, MID[3] = {2, 0, 1}, LEAF[3] = {1, 2, 0};
    for (int m = 0; m < 3; ++m) {
        t->mode[m].root = ROOT[m];
        t->mode[m].mid = MID[m];
        t->mode[m].leaf = LEAF[m];
    }
    std::vector<uint2> heads[3];
    if (n == 0) {
        t->normsq = 0.0;
        for (int m = 0; m < 3; ++m)
            build_mode(ctx, t, m, nullptr, nullptr, nullptr, nullptr, 0, heads[m]);
        return;
    }
    // coordinates and values are checked here and the outcome read with the
    // distinct count below: until then only sort keys (any bits) and
    // permutation-indexed copies depend on them
    uint32_t *flag = sc.alloc<uint32_t>(1);
    DF_HIP(hipMemsetAsync(flag, 0, sizeof(uint32_t), s));
    hipLaunchKernelGGL(k_validate, dim3(grid_for(n)), dim3(kThreads), 0, s, d_i, d_j, d_k, d_val,
                       n, (uint32_t)t->dims[0], (uint32_t)t->dims[1], (uint32_t)t->dims[2], flag);
    DF_LAUNCHED();
    const int bI = bits_for(t->dims[0]), bJ = bits_for(t->dims[1]), bK = bits_for(t->dims[2]);
    uint64_t *key = sc.alloc<uint64_t>(n), *kalt = sc.alloc<uint64_t>(n);
    uint32_t *perm = sc.alloc<uint32_t>(n), *palt = sc.alloc<uint32_t>(n);
    hipLaunchKernelGGL(k_iota, dim3(grid_for(n)), dim3(kThreads), 0, s, perm, n);
    // mode-0 order (i, k, j)
    if (bI + bK + bJ <= 64) {
        hipLaunchKernelGGL(k_make_key, dim3(grid_for(n)), dim3(kThreads), 0, s, key, d_i, bK + bJ,
                           d_k, bJ, d_j, (const uint32_t *)nullptr, n);
        radix_sort(key, perm, kalt, palt, n, bI + bK + bJ, sc, s);
    } else {
        hipLaunchKernelGGL(k_make_key, dim3(grid_for(n)), dim3(kThreads), 0, s, key,
                           (const uint32_t *)nullptr, 0, (const uint32_t *)nullptr, 0, d_j,
                           (const uint32_t *)nullptr, n);
        radix_sort(key, perm, kalt, palt, n, bJ, sc, s);
        hipLaunchKernelGGL(k_make_key, dim3(grid_for(n)), dim3(kThreads), 0, s, key, d_i, bK, d_k,
                           0, (const uint32_t *)nullptr, (const uint32_t *)perm, n);
        radix_sort(key, perm, kalt, palt, n, bI + bK, sc, s);
    }
    sc.release(key);
    sc.release(kalt);
    // gather into sorted coordinates and merge duplicates
    uint32_t *si = sc.alloc<uint32_t>(n), *sj = sc.alloc<uint32_t>(n), *sk = sc.alloc<uint32_t>(n);
    float *sv = sc.alloc<float>(n);
    hipLaunchKernelGGL(k_gather4, dim3(grid_for(n)), dim3(kThreads), 0, s, perm, n, d_i, d_j, d_k,
                       d_val, si, sj, sk, sv);
    uint32_t *dflag = perm, *dpos = palt;  // reuse
    hipLaunchKernelGGL(k_distinct_flags, dim3(grid_for(n)), dim3(kThreads), 0, s, si, sj, sk, n,
                       dflag);
    scan_exclusive_u32(dflag, dpos, n, s, &sc.mem);
    uint32_t h[3];
    DF_HIP(hipMemcpyAsync(&h[0], flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    DF_HIP(hipMemcpyAsync(&h[1], dpos + n - 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    DF_HIP(hipMemcpyAsync(&h[2], dflag + n - 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    DF_HIP(hipStreamSynchronize(s));
    if (h[0] & 1u) throw Error{DFACTO_E_RANGE, "a coordinate is not below its dimension"};
    if (h[0] & 2u) throw Error{DFACTO_E_NUMERIC, "a tensor value is NaN or Inf"};
    const int64_t nd = (int64_t)h[1] + h[2];
    uint32_t *di = sc.alloc<uint32_t>(nd), *dj = sc.alloc<uint32_t>(nd), *dk = sc.alloc<uint32_t>(nd);
    float *dv = sc.alloc<float>(nd);
    hipLaunchKernelGGL(k_merge_runs, dim3(grid_for(n)), dim3(kThreads), 0, s, dflag, dpos, n, si,
                       sj, sk, sv, di, dj, dk, dv);
    DF_LAUNCHED();
    sc.release(si);
    sc.release(sj);
    sc.release(sk);
    sc.release(sv);
    t->nnz = nd;
    // ||X||^2 in FP64, fixed reduction order
    {
        const unsigned nb = std::min<unsigned>(grid_for(nd), 1024u);
        double *part = sc.alloc<double>(nb), *tot = sc.alloc<double>(1);
        hipLaunchKernelGGL(k_sumsq_partial, dim3(nb), dim3(kThreads), 0, s, dv, nd, part);
        hipLaunchKernelGGL(k_sum_f64_final, dim3(1), dim3(kThreads), 0, s, part, (int)nb, tot);
        // lands when build_tensor waits for the stream at its end
        DF_HIP(hipMemcpyAsync(&t->normsq, tot, sizeof(double), hipMemcpyDeviceToHost, s));
    }
    // mode 0: already in (i, k, j) order
    build_mode(ctx, t, 0, di, dk, dj, dv, nd, heads[0]);
    // modes 1 and 2: stable sort by (root, mid) from the mode-0 order
    uint64_t *key2 = sc.alloc<uint64_t>(nd), *kalt2 = sc.alloc<uint64_t>(nd);
    uint32_t *p2 = perm, *palt2 = palt;  // n >= nd
    uint32_t *gr = sc.alloc<uint32_t>(nd), *gm = sc.alloc<uint32_t>(nd), *gl = sc.alloc<uint32_t>(nd);
    float *gv = sc.alloc<float>(nd);
    const uint32_t *coord[3] = {di, dj, dk};
    const int bits[3] = {bI, bJ, bK};
    for (int m = 1; m < 3; ++m) {
        const ModeData &md = t->mode[m];
        hipLaunchKernelGGL(k_iota, dim3(grid_for(nd)), dim3(kThreads), 0, s, p2, nd);
        hipLaunchKernelGGL(k_make_key, dim3(grid_for(nd)), dim3(kThreads), 0, s, key2,
                           coord[md.root], bits[md.mid], coord[md.mid], 0,
                           (const uint32_t *)nullptr, (const uint32_t *)nullptr, nd);
        radix_sort(key2, p2, kalt2, palt2, nd, bits[md.root] + bits[md.mid], sc, s);
        hipLaunchKernelGGL(k_gather4, dim3(grid_for(nd)), dim3(kThreads), 0, s, p2, nd,
                           coord[md.root], coord[md.mid], coord[md.leaf], dv, gr, gm, gl, gv);
        DF_LAUNCHED();
        build_mode(ctx, t, m, gr, gm, gl, gv, nd, heads[m]);
    }
    DF_HIP(hipStreamSynchronize(s));  // the chunk heads, ||X||^2
    for (int m = 0; m < 3; ++m) finish_runs(t, t->mode[m], s, heads[m]);
    DF_HIP(hipStreamSynchronize(s));  // the run lists' uploads
}

}  // namespace dfacto
