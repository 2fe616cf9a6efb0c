// dense.hip -- the small dense FP64 parts of CP-ALS and GD (Appendix B and C)
//
//  * Gram F^T F of a factor or of an MTTKRP result, FP64 accumulation: on
//    the matrix cores (FP64 MFMA) for R <= 64, else register-tiled 8x8 outer
//    products per thread; then a fixed-order reduction over blocks.
//  * H = G_p * G_q + reg I (Appendix A: (A kr B)^T (A kr B) = A^T A * B^T B,
//    ridge term of the regularized update).
//  * One-workgroup FP64 solve: Cholesky inverse of H, or the Moore-Penrose
//    pseudo-inverse from a parallel cyclic Jacobi eigen-decomposition when a
//    pivot shows H is numerically singular.  Working set in LDS when small.
//  * Column norms, the new Gram and the fit from R x R algebra: with
//    Fhat = M H^-1,  Fhat^T Fhat = H^-1 (M^T M) H^-1, so
//    lambda_r^2 = [H^-1 M^T M H^-1]_rr and  <X, Xhat> = <Fhat, M> =
//    trace(H^-1 M^T M) for the last mode; ||Xhat||^2 = lambda^T (G_A * G_B *
//    G_C) lambda.
//  * Row maps F = M W (W = H^-1 diag(1/lambda)) and the GD gradient
//    -M + F H over LDS-staged row tiles, the R x R matrix broadcast from LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <type_traits>

#include "internal.hpp"

namespace dfacto {
namespace {

constexpr int kBlock = 256;

template <typename T>
__device__ __forceinline__ double ld(const T *p, int64_t i);
template <>
__device__ __forceinline__ double ld<float>(const float *p, int64_t i) {
    return (double)p[i];
}
template <>
__device__ __forceinline__ double ld<uint16_t>(const uint16_t *p, int64_t i) {
    return (double)__uint_as_float((uint32_t)p[i] << 16);
}

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t b = __float_as_uint(f);
    if ((b & 0x7F800000u) == 0x7F800000u) return (uint16_t)((b >> 16) | ((b & 0xFFFFu) ? 0x40u : 0u));
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

template <typename T>
__device__ __forceinline__ void st_out(T *p, int64_t i, double v);
template <>
__device__ __forceinline__ void st_out<float>(float *p, int64_t i, double v) {
    p[i] = (float)v;
}
template <>
__device__ __forceinline__ void st_out<uint16_t>(uint16_t *p, int64_t i, double v) {
    p[i] = f32_to_bf16((float)v);
}

// 8 consecutive entries p[base + c0 .. + 8) widened to double; entries at
// columns >= R read as 0.  Vector loads when the row layout allows.
// `vec` (computed on the host) says the rows allow 16-byte loads: R is a
// multiple of 4 (FP32) or 8 (BF16) and the base pointer is 16-byte aligned.
template <typename T>
__device__ __forceinline__ void load8(const T *p, int64_t base, int c0, int R, bool vec,
                                      double (&v)[8]);
template <>
__device__ __forceinline__ void load8<float>(const float *p, int64_t base, int c0, int R, bool vec,
                                             double (&v)[8]) {
    if (vec && c0 + 8 <= R) {
        const float4 a = *reinterpret_cast<const float4 *>(p + base + c0);
        const float4 b = *reinterpret_cast<const float4 *>(p + base + c0 + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = (c0 + q < R) ? (double)p[base + c0 + q] : 0.0;
    }
}
template <>
__device__ __forceinline__ void load8<uint16_t>(const uint16_t *p, int64_t base, int c0, int R,
                                                bool vec, double (&v)[8]) {
    if (vec && c0 + 8 <= R) {
        const uint4 a = *reinterpret_cast<const uint4 *>(p + base + c0);
        const uint32_t w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v[2 * q] = (double)__uint_as_float(w[q] << 16);
            v[2 * q + 1] = (double)__uint_as_float(w[q] & 0xFFFF0000u);
        }
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q)
            v[q] = (c0 + q < R) ? (double)__uint_as_float((uint32_t)p[base + c0 + q] << 16) : 0.0;
    }
}

// ---------------------------------------------------------------------------
// Gram: part[b][r][s] = sum over the rows visited by block b of F[row][r] F[row][s]
// grid.x: row blocks, grid.y: TSxTS output tiles.  A tile is covered by
// (TS/8)^2 threads with 8x8 register tiles; the block holds kBlock/(TS/8)^2
// slices of rows, combined in slice order through LDS.
// ---------------------------------------------------------------------------
template <typename T, int TS>
__global__ __launch_bounds__(kBlock) void k_gram_partial(const T *__restrict__ F, int64_t rows,
                                                         int R, int vec, double *__restrict__ part) {
    constexpr int TT = TS / 8;
    constexpr int TPT = TT * TT;
    constexpr int SL = kBlock / TPT;
    __shared__ double tile[TS * TS];
    const int nt = (R + TS - 1) / TS;
    const int rt = blockIdx.y / nt, ct = blockIdx.y % nt;
    const int slice = threadIdx.x / TPT, t = threadIdx.x % TPT;
    const int ty = t / TT, tx = t % TT;
    const int ra = rt * TS + ty * 8, cb = ct * TS + tx * 8;
    double acc[8][8];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 8; ++b) acc[a][b] = 0.0;
    const bool active = ra < R && cb < R;
    if (active) {
        for (int64_t row = (int64_t)blockIdx.x * SL + slice; row < rows;
             row += (int64_t)gridDim.x * SL) {
            double x[8], y[8];
            load8<T>(F, row * R, ra, R, vec, x);
            load8<T>(F, row * R, cb, R, vec, y);
#pragma unroll
            for (int a = 0; a < 8; ++a)
#pragma unroll
                for (int b = 0; b < 8; ++b) acc[a][b] = fma(x[a], y[b], acc[a][b]);
        }
    }
    for (int s = 0; s < SL; ++s) {
        __syncthreads();
        if (slice == s) {
#pragma unroll
            for (int a = 0; a < 8; ++a)
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const int e = (ty * 8 + a) * TS + tx * 8 + b;
                    tile[e] = (s == 0) ? acc[a][b] : tile[e] + acc[a][b];
                }
        }
    }
    __syncthreads();
    double *pb = part + (size_t)blockIdx.x * R * R;
    for (int e = threadIdx.x; e < TS * TS; e += kBlock) {
        const int r = rt * TS + e / TS, c = ct * TS + e % TS;
        if (r < R && c < R) pb[r * R + c] = tile[e];
    }
}

// Gram on the matrix cores: v_mfma_f64_16x16x4f64 multiplies a 16x4 by a
// 4x16 FP64 tile.  For F^T F, a step covers 4 rows: lane l supplies
// F[k0 + l/16][16 t + l%16] for each 16-column tile t, as the A operand
// (F^T, tile rt) and the B operand (F, tile ct); the 16x16 result D holds
// D[l/16 + 4 i][l%16] in accumulator element i of lane l (checked on the
// device against an encoded product).  Only tile pairs
// rt <= ct are computed; the lower triangle is written as their mirror.
// Each wave walks its rows 16 at a time; the waves of a block are combined
// in a fixed order through LDS.  R <= 64 (at most 4 column tiles).
typedef double double4v __attribute__((ext_vector_type(4)));
constexpr int kMfmaMaxTiles = 4;

// NT consecutive entries F[row][c0 .. c0 + NT) as FP32 bit patterns (a BF16
// value is its FP32 pattern with the low half zero), zero past the last row
// or column.  VEC: R == 16 NT and the rows are aligned for one NT-element
// vector load.
// the FP32 bits of element i (BF16: its bits in the upper half)
__device__ __forceinline__ uint32_t gram_bits(const DF_GLOBAL float *F, int64_t i) {
    return __float_as_uint(F[i]);
}
__device__ __forceinline__ uint32_t gram_bits(const DF_GLOBAL uint16_t *F, int64_t i) {
    return (uint32_t)F[i] << 16;
}

// F through a global-space pointer (the grouped kernels read it from a
// descriptor: plain loads would be flat ones, whose waits also cover the
// loads issued for the next steps)
template <typename T, int NT, bool VEC>
__device__ __forceinline__ void gram_load(const T *__restrict__ F_, int64_t row, int64_t rows,
                                          int R, int c0, uint32_t (&v)[NT]) {
    const DF_GLOBAL T *F = gptr(F_);
    if (VEC && NT == 2) {
        if (row < rows) {
            if constexpr (sizeof(T) == 4) {
                const df_u2 a = *reinterpret_cast<const DF_GLOBAL df_u2 *>(F + row * R + c0);
                v[0] = a.x;
                v[1] = a.y;
            } else {
                const uint32_t a = *reinterpret_cast<const DF_GLOBAL uint32_t *>(F + row * R + c0);
                v[0] = a << 16;
                v[1] = a & 0xFFFF0000u;
            }
        } else {
            v[0] = v[1] = 0u;
        }
        return;
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
        v[t] = (row < rows && c0 + t < R) ? gram_bits(F, row * R + c0 + t) : 0u;
}

// Block b of nb: the launch's own block, or a grouped launch's virtual one.
template <typename T, int NT, int BS, bool VEC>
__device__ __forceinline__ void gram_mfma_body(const T *__restrict__ F, int64_t rows, int R,
                                               double *__restrict__ part, uint32_t b,
                                               uint32_t nb) {
    constexpr int NP = NT * (NT + 1) / 2;  // tile pairs rt <= ct
    constexpr int NW = BS / 64;            // waves per block
    // steps loaded per batch: the next batch's loads are in flight while the
    // current one's MFMAs run (a wave takes only a few dozen steps, so one
    // step ahead leaves the loop waiting on memory); one step for R > 32,
    // where a second would cost occupancy
    constexpr int PD = NT <= 2 ? 2 : 1;
    __shared__ double sacc[NP * 256];
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int kr = lane / 16, cl = lane % 16;
    double4v acc[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) acc[q] = double4v{0.0, 0.0, 0.0, 0.0};
    const int64_t nwaves = (int64_t)nb * NW;
    const int64_t gw = (int64_t)b * NW + wave;
    // rows [16 * step, 16 * step + 16) for step = gw, gw + nwaves, ... in
    // that order; rows past the end read as zero.
    const int64_t nsteps = (rows + 15) / 16;
    // Column tile t, MFMA index c is column c * NT + t, so a lane reads the
    // NT consecutive columns cl * NT .. + NT of a row.
    auto load = [&](int64_t s0, uint32_t (&v)[PD][4][NT]) {
#pragma unroll
        for (int p = 0; p < PD; ++p)
#pragma unroll
            for (int sub = 0; sub < 4; ++sub)
                gram_load<T, NT, VEC>(F, (s0 + p * nwaves) * 16 + sub * 4 + kr, rows, R, cl * NT,
                                      v[p][sub]);
    };
    uint32_t v[PD][4][NT];
    if (gw < nsteps) load(gw, v);
    for (int64_t s0 = gw; s0 < nsteps; s0 += PD * nwaves) {
        uint32_t vn[PD][4][NT];
        load(s0 + PD * nwaves, vn);
#pragma unroll
        for (int p = 0; p < PD; ++p) {
            if (s0 + p * nwaves >= nsteps) continue;  // uniform across the wave
#pragma unroll
            for (int sub = 0; sub < 4; ++sub) {
                double x[NT];
#pragma unroll
                for (int t = 0; t < NT; ++t) x[t] = (double)__uint_as_float(v[p][sub][t]);
                int q = 0;
#pragma unroll
                for (int rt = 0; rt < NT; ++rt)
#pragma unroll
                    for (int ct = rt; ct < NT; ++ct, ++q)
                        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[rt], x[ct], acc[q], 0, 0, 0);
            }
        }
#pragma unroll
        for (int p = 0; p < PD; ++p)
#pragma unroll
            for (int sub = 0; sub < 4; ++sub)
#pragma unroll
                for (int t = 0; t < NT; ++t) v[p][sub][t] = vn[p][sub][t];
    }
    // combine the waves of the block in wave order
    for (int w = 0; w < NW; ++w) {
        if (wave == w) {
#pragma unroll
            for (int q = 0; q < NP; ++q)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int e = q * 256 + (kr + 4 * i) * 16 + cl;
                    sacc[e] = (w == 0) ? acc[q][i] : sacc[e] + acc[q][i];
                }
        }
        __syncthreads();
    }
    DF_GLOBAL double *pb = gptr(part) + (size_t)b * R * R;
    for (int e = threadIdx.x; e < NP * 256; e += BS) {
        int q = e / 256, rt = 0;
        while (q >= NT - rt) { q -= NT - rt; ++rt; }  // pair index -> (rt, ct)
        const int ct = rt + q;
        const int r = ((e % 256) / 16) * NT + rt, c = (e % 16) * NT + ct;
        if (r < R && c < R) {
            pb[r * R + c] = sacc[e];
            if (rt != ct) pb[c * R + r] = sacc[e];
        }
    }
}

template <typename T, int NT, int BS, bool VEC>
__global__ __launch_bounds__(BS) void k_gram_mfma(const T *__restrict__ F, int64_t rows, int R,
                                                  double *__restrict__ part) {
    gram_mfma_body<T, NT, BS, VEC>(F, rows, R, part, blockIdx.x, gridDim.x);
}

template <typename T, int NT, int BS, bool VEC>
__global__ __launch_bounds__(BS) void k_gram_mfma_group(const GramJob *__restrict__ jobs,
                                                        const uint2 *__restrict__ vb) {
    const uint2 v = vb[blockIdx.x];
    const GramJob &j = jobs[v.x];
    gram_mfma_body<T, NT, BS, VEC>((const T *)j.F, j.rows, j.R, j.part, v.y, j.nblk);
}

// G[e] = sum_b part[b][e]: a block takes 16 entries; slice q (16 per entry)
// sums the partials b = q, q + 16, ...; the slices are combined in order.
// The first 16 partials of a slice are loaded together, then added in order.
__device__ __forceinline__ void gram_reduce_body(const double *__restrict__ part_, int nblk, int R,
                                                 double *__restrict__ G_, uint32_t b) {
    const DF_GLOBAL double *part = gptr(part_);
    DF_GLOBAL double *G = gptr(G_);
    __shared__ double sh[16][17];
    const int e = b * 16 + threadIdx.x % 16;
    const int sl = threadIdx.x / 16;
    const int RR = R * R;
    double s = 0.0;
    if (e < RR) {
        double x[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int pb = sl + 16 * u;
            x[u] = pb < nblk ? part[(size_t)pb * RR + e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u)
            if (sl + 16 * u < nblk) s += x[u];
        for (int pb = sl + 256; pb < nblk; pb += 16) s += part[(size_t)pb * RR + e];
    }
    sh[sl][threadIdx.x % 16] = s;
    __syncthreads();
    if (threadIdx.x < 16 && e < RR) {
        double t = sh[0][threadIdx.x];
#pragma unroll
        for (int q = 1; q < 16; ++q) t += sh[q][threadIdx.x];
        G[e] = t;
    }
}

__global__ __launch_bounds__(kBlock) void k_gram_reduce(const double *__restrict__ part, int nblk,
                                                        int R, double *__restrict__ G) {
    gram_reduce_body(part, nblk, R, G, blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_gram_reduce_group(const GramJob *__restrict__ jobs,
                                                              const uint2 *__restrict__ vb) {
    const uint2 v = vb[blockIdx.x];
    const GramJob &j = jobs[v.x];
    gram_reduce_body(j.part, (int)j.nblk, j.R, j.G, v.y);
}

__global__ void k_hadamard(int R, const double *__restrict__ Gp, const double *__restrict__ Gq,
                           double reg, double *__restrict__ H) {
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= R * R) return;
    H[e] = Gp[e] * Gq[e] + ((e / R == e % R) ? reg : 0.0);
}

// fixed-order block reduction of one double per thread
__device__ double block_sum(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__device__ double block_max(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// R x R working matrices live in LDS up to these ranks (at most ~56 KB of
// dynamic LDS), else in global scratch.
constexpr int kSolveSmemMaxR = 44;   // 3 R^2 doubles
constexpr int kLambdaSmemMaxR = 40;  // 4 R^2 + R doubles

// ---------------------------------------------------------------------------
// one-workgroup solve.  Working set: 3 R^2 doubles (H, A, B / V), in
// dynamic LDS when SMEM, else in `scratch`.  flag[0] = 1 when the
// pseudo-inverse path was taken.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Gauss-Jordan on [H | I] in the registers of one wave (R <= 32): lane l
// holds column l of the R x 2R working matrix; the pivot and the pivot
// column's entries reach every lane by readlane.  The arithmetic (scale the
// pivot row by 1/pivot, then row_i -= a_ij * row_j) is the same, operation
// for operation, as the LDS version in k_solve.  On success columns R .. 2R-1
// (H^-1) are written to Bw (R x R, row-major); returns false at the first
// pivot that is not above tol.
template <int B, int E, typename Fn>
__device__ __forceinline__ void unroll_for(Fn &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        unroll_for<B + 1, E>(f);
    }
}

__device__ bool gauss_jordan_wave(const double *H, int R, double tol, double *Bw) {
    constexpr int RM = 32;
    const int l = threadIdx.x % 64;
    double col[RM];
#pragma unroll
    for (int i = 0; i < RM; ++i)
        col[i] = (i < R) ? (l < R ? H[i * R + l] : (l - R == i ? 1.0 : 0.0)) : 0.0;
    bool ok = true;
    // j and i are compile-time constants, so col[] stays in registers
    unroll_for<0, RM>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if (!ok || j >= R) return;
        const double piv = readlane_f64(col[j], j);
        if (!(piv > tol)) {
            ok = false;
            return;
        }
        const double inv = 1.0 / piv;
        col[j] *= inv;
        unroll_for<0, RM>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            if (i == j || i >= R) return;
            col[i] = fma(-readlane_f64(col[i], j), col[j], col[i]);
        });
        __builtin_amdgcn_sched_barrier(0);  // keep the steps apart: no hoisted readlanes
    });
    if (!ok) return false;
    if (l >= R && l < 2 * R) {
#pragma unroll
        for (int i = 0; i < RM; ++i)
            if (i < R) Bw[i * R + (l - R)] = col[i];
    }
    return true;
}

template <bool SMEM>
__device__ void solve_body(int R, const double *__restrict__ Gp, const double *__restrict__ Gq,
                           double reg, double *__restrict__ Hinv, double *__restrict__ scratch,
                           int *flag, double *dyn) {
    __shared__ double sh[kBlock];
    __shared__ int s_fail;
    __shared__ double s_c[kBlock], s_s[kBlock];
    __shared__ int s_p[kBlock], s_q[kBlock];
    const int tid = threadIdx.x;
    const int RR = R * R;
    double *base = SMEM ? dyn : scratch;
    double *H = base, *L = base + RR, *Li = base + 2 * RR;
    for (int e = tid; e < RR; e += kBlock) {
        H[e] = Gp[e] * Gq[e] + ((e / R == e % R) ? reg : 0.0);
        L[e] = 0.0;
        Li[e] = 0.0;
    }
    __syncthreads();
    double dm = 0.0;
    for (int r = tid; r < R; r += kBlock) dm = fmax(dm, H[r * R + r]);
    const double dmax = block_max(dm, sh);
    const double tol = (double)R * DBL_EPSILON * dmax;
    if (tid == 0) s_fail = (dmax > 0.0) ? 0 : 1;
    __syncthreads();
    // Gauss-Jordan on [H | I] without pivoting (H is symmetric): the pivot at
    // step j is the Schur-complement diagonal d_j = L_jj^2 of the Cholesky
    // factorization H = L L^T, so "every d_j > R eps max diag(H)" is the
    // Cholesky test for a numerically positive definite H.  If it fails, the
    // pseudo-inverse below is used instead.  Aw (in L) is the working copy of
    // H, Bw (in Li) starts as I and ends as H^-1.
    double *Aw = L, *Bw = Li;
    __shared__ double s_f[kBlock];
    if (R <= 32) {
        if (tid < 64 && !s_fail) {
            const bool ok = gauss_jordan_wave(H, R, tol, Bw);
            if (tid == 0 && !ok) s_fail = 1;
        }
        __syncthreads();
    } else {
        for (int e = tid; e < RR; e += kBlock) {
            Aw[e] = H[e];
            Bw[e] = (e / R == e % R) ? 1.0 : 0.0;
        }
        __syncthreads();
        for (int j = 0; j < R; ++j) {
            const double piv = Aw[j * R + j];
            if (!(piv > tol)) {  // uniform: every thread reads the same value
                if (tid == 0) s_fail = 1;
                break;
            }
            const double inv = 1.0 / piv;
            __syncthreads();  // all threads have read the pivot
            for (int k = tid; k < 2 * R; k += kBlock) {
                if (k < R) Aw[j * R + k] *= inv;
                else Bw[j * R + k - R] *= inv;
            }
            for (int i = tid; i < R; i += kBlock) s_f[i] = (i == j) ? 0.0 : Aw[i * R + j];
            __syncthreads();
            for (int e = tid; e < R * 2 * R; e += kBlock) {
                const int i = e / (2 * R), k = e % (2 * R);
                const double f = s_f[i];
                if (f == 0.0) continue;
                if (k < R) Aw[i * R + k] = fma(-f, Aw[j * R + k], Aw[i * R + k]);
                else Bw[i * R + k - R] = fma(-f, Bw[j * R + k - R], Bw[i * R + k - R]);
            }
            __syncthreads();
        }
    }
    __syncthreads();
    if (!s_fail) {
        for (int e = tid; e < RR; e += kBlock) {
            const int r = e / R, c = e % R;
            Hinv[e] = 0.5 * (Bw[r * R + c] + Bw[c * R + r]);
        }
        if (tid == 0) flag[0] = 0;
        return;
    }
    // pseudo-inverse: parallel cyclic Jacobi on A = H, V = I
    double *A = L, *V = Li;
    for (int e = tid; e < RR; e += kBlock) {
        A[e] = H[e];
        V[e] = (e / R == e % R) ? 1.0 : 0.0;
    }
    __syncthreads();
    const int n2 = (R + 1) & ~1;  // players in the round-robin schedule
    const int npair = n2 / 2;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int e = tid; e < RR; e += kBlock) {
            const double a2 = A[e] * A[e];
            tot += a2;
            if (e / R != e % R) off += a2;
        }
        off = block_sum(off, sh);
        tot = block_sum(tot, sh);
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int round = 0; round < n2 - 1; ++round) {
            for (int pi = tid; pi < npair; pi += kBlock) {
                auto player = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + round) % (n2 - 1); };
                int p = player(pi), q = player(n2 - 1 - pi);
                if (p > q) { const int t = p; p = q; q = t; }
                double c = 1.0, s = 0.0;
                if (q < R) {
                    const double apq = A[p * R + q];
                    if (apq != 0.0) {
                        const double theta = (A[q * R + q] - A[p * R + p]) / (2.0 * apq);
                        const double t = (theta >= 0 ? 1.0 : -1.0) /
                                         (fabs(theta) + sqrt(theta * theta + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        s = t * c;
                    }
                }
                s_p[pi] = p;
                s_q[pi] = q;
                s_c[pi] = c;
                s_s[pi] = s;
            }
            __syncthreads();
            // A <- A J and V <- V J (columns p, q of every disjoint pair)
            for (int e = tid; e < npair * R; e += kBlock) {
                const int pi = e / R, k = e % R;
                const int p = s_p[pi], q = s_q[pi];
                if (q >= R || s_s[pi] == 0.0) continue;
                const double c = s_c[pi], s = s_s[pi];
                const double akp = A[k * R + p], akq = A[k * R + q];
                A[k * R + p] = c * akp - s * akq;
                A[k * R + q] = s * akp + c * akq;
                const double vkp = V[k * R + p], vkq = V[k * R + q];
                V[k * R + p] = c * vkp - s * vkq;
                V[k * R + q] = s * vkp + c * vkq;
            }
            __syncthreads();
            // A <- J^T A (rows p, q)
            for (int e = tid; e < npair * R; e += kBlock) {
                const int pi = e / R, k = e % R;
                const int p = s_p[pi], q = s_q[pi];
                if (q >= R || s_s[pi] == 0.0) continue;
                const double c = s_c[pi], s = s_s[pi];
                const double apk = A[p * R + k], aqk = A[q * R + k];
                A[p * R + k] = c * apk - s * aqk;
                A[q * R + k] = s * apk + c * aqk;
            }
            __syncthreads();
        }
    }
    double wm = 0.0;
    for (int r = tid; r < R; r += kBlock) wm = fmax(wm, A[r * R + r]);
    const double wmax = block_max(wm, sh);
    const double wtol = (double)R * DBL_EPSILON * wmax;
    for (int e = tid; e < RR; e += kBlock) {
        const int r = e / R, s = e % R;
        double acc = 0.0;
        for (int k = 0; k < R; ++k) {
            const double w = A[k * R + k];
            if (w > wtol) acc += V[r * R + k] * V[s * R + k] / w;
        }
        Hinv[e] = acc;
    }
    if (tid == 0) flag[0] = 1;
}

template <bool SMEM>
__global__ __launch_bounds__(kBlock) void k_solve(int R, const double *__restrict__ Gp,
                                                  const double *__restrict__ Gq, double reg,
                                                  double *__restrict__ Hinv,
                                                  double *__restrict__ scratch, int *flag) {
    extern __shared__ double dyn[];
    solve_body<SMEM>(R, Gp, Gq, reg, Hinv, scratch, flag, dyn);
}

template <bool SMEM>
__global__ __launch_bounds__(kBlock) void k_solve_group(const SolveJob *__restrict__ jobs) {
    extern __shared__ double dyn[];
    const SolveJob &j = jobs[blockIdx.x];
    solve_body<SMEM>(j.R, j.Gp, j.Gq, j.reg, j.Hinv, j.scratch, j.flag, dyn);
}

// ---------------------------------------------------------------------------
// lambda, new Gram, W and (last mode) fit -- one workgroup.  Working set:
// Hinv, MtM, T1 = MtM Hinv, S = Hinv T1 (4 R^2) and lambda (R), in dynamic
// LDS when SMEM, else in `scratch`.
// ---------------------------------------------------------------------------
template <bool SMEM>
__device__ void als_lambda_body(int R, int mode, const double *__restrict__ Hinv_g,
                                const double *__restrict__ MtM_g, double *__restrict__ Gn,
                                double *__restrict__ W, double *__restrict__ lambda_out,
                                const double *__restrict__ GA, const double *__restrict__ GB,
                                double normsq, double *__restrict__ fit_out,
                                double *__restrict__ scratch, double *dyn) {
    __shared__ double sh[kBlock];
    const int tid = threadIdx.x;
    const int RR = R * R;
    double *base = SMEM ? dyn : scratch;
    double *Hi = base, *MM = base + RR, *T1 = base + 2 * RR, *S = base + 3 * RR,
           *lam = base + 4 * RR;
    for (int e = tid; e < RR; e += kBlock) {
        Hi[e] = Hinv_g[e];
        MM[e] = MtM_g[e];
    }
    __syncthreads();
    for (int e = tid; e < RR; e += kBlock) {
        const int r = e / R, s = e % R;
        double acc = 0.0;
        for (int k = 0; k < R; ++k) acc += MM[r * R + k] * Hi[k * R + s];
        T1[e] = acc;
    }
    __syncthreads();
    for (int e = tid; e < RR; e += kBlock) {
        const int r = e / R, s = e % R;
        double acc = 0.0;
        for (int k = 0; k < R; ++k) acc += Hi[r * R + k] * T1[k * R + s];
        S[e] = acc;
    }
    __syncthreads();
    for (int r = tid; r < R; r += kBlock) {
        const double d = S[r * R + r];
        lam[r] = d > 0.0 ? sqrt(d) : 0.0;
        lambda_out[r] = lam[r];
    }
    __syncthreads();
    double in = 0.0, xh = 0.0;
    for (int e = tid; e < RR; e += kBlock) {
        const int r = e / R, s = e % R;
        const double lr = lam[r], ls = lam[s];
        const double g = (lr > 0.0 && ls > 0.0) ? S[e] / (lr * ls) : 0.0;
        Gn[e] = g;
        W[e] = ls > 0.0 ? Hi[e] / ls : 0.0;
        if (mode == 2) {
            in += Hi[e] * MM[e];
            xh += lr * ls * GA[e] * GB[e] * g;
        }
    }
    if (mode != 2) return;
    in = block_sum(in, sh);
    xh = block_sum(xh, sh);
    if (tid == 0) {
        double res2 = normsq + xh - 2.0 * in;
        if (res2 < 0.0) res2 = 0.0;
        *fit_out = normsq > 0.0 ? 1.0 - sqrt(res2) / sqrt(normsq) : 0.0;
    }
}

// ---------------------------------------------------------------------------
// Fit from the STORED last factor (BF16 storage): the rounded factor C that
// later calls read differs from M H^-1 diag(1/lambda), so the fit is formed
// from C itself, as for the other two factors whose Grams are re-formed
// from their stored values:
//   <X, Xhat> = sum_r lambda_r sum_k C[k, r] M[k, r]   (M: mode-2 MTTKRP)
//   ||Xhat||^2 = lambda^T (G_A * G_B * G_C) lambda     (G_C from stored C)
// Partial sums of the weighted inner product per block (fit_blocks of them,
// each a fixed-order strided sum), then one block finishes.
// ---------------------------------------------------------------------------
template <typename T>
__device__ void wdot_body(const T *__restrict__ F, const float *__restrict__ X, int64_t rows,
                          int R, const double *__restrict__ lam, uint32_t b, uint32_t nb,
                          double *__restrict__ part, double *sh, double *sl) {
    for (int r = threadIdx.x; r < R; r += kBlock) sl[r] = lam[r];
    __syncthreads();
    const int64_t n = rows * (int64_t)R;
    const int64_t S = (int64_t)nb * kBlock;
    int64_t e = (int64_t)b * kBlock + threadIdx.x;
    int r = (int)(e % R);
    const int dr = (int)(S % R);
    double acc = 0.0;
    for (; e < n; e += S) {
        acc = fma(sl[r] * ld<T>(F, e), (double)X[e], acc);
        r += dr;
        if (r >= R) r -= R;
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) part[b] = acc;
}

__device__ void fit_finish_body(int R, const double *__restrict__ lam,
                                const double *__restrict__ GA, const double *__restrict__ GB,
                                const double *__restrict__ GC, const double *__restrict__ part,
                                uint32_t npart, double normsq, double *__restrict__ fit,
                                double *sh) {
    double in = 0.0, xh = 0.0;
    for (uint32_t b = threadIdx.x; b < npart; b += kBlock) in += part[b];
    for (int e = threadIdx.x; e < R * R; e += kBlock) {
        const int r = e / R, s = e % R;
        xh += lam[r] * lam[s] * GA[e] * GB[e] * GC[e];
    }
    in = block_sum(in, sh);
    xh = block_sum(xh, sh);
    if (threadIdx.x == 0) {
        double res2 = normsq + xh - 2.0 * in;
        if (res2 < 0.0) res2 = 0.0;
        *fit = normsq > 0.0 ? 1.0 - sqrt(res2) / sqrt(normsq) : 0.0;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_wdot(const T *__restrict__ F,
                                                 const float *__restrict__ X, int64_t rows, int R,
                                                 const double *__restrict__ lam,
                                                 double *__restrict__ part) {
    __shared__ double sh[kBlock], sl[DFACTO_MAX_R];
    wdot_body<T>(F, X, rows, R, lam, blockIdx.x, gridDim.x, part, sh, sl);
}

__global__ __launch_bounds__(kBlock) void k_fit_finish(int R, const double *__restrict__ lam,
                                                       const double *__restrict__ GA,
                                                       const double *__restrict__ GB,
                                                       const double *__restrict__ GC,
                                                       const double *__restrict__ part,
                                                       uint32_t npart, double normsq,
                                                       double *__restrict__ fit) {
    __shared__ double sh[kBlock];
    fit_finish_body(R, lam, GA, GB, GC, part, npart, normsq, fit, sh);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_wdot_group(const FitJob *__restrict__ jobs,
                                                       const uint2 *__restrict__ items) {
    __shared__ double sh[kBlock], sl[DFACTO_MAX_R];
    const uint2 v = items[blockIdx.x];
    const FitJob &j = jobs[v.x];
    wdot_body<T>((const T *)j.F, j.M, j.rows, j.R, j.lambda, v.y, j.nblk, j.part, sh, sl);
}

__global__ __launch_bounds__(kBlock) void k_fit_finish_group(const FitJob *__restrict__ jobs) {
    __shared__ double sh[kBlock];
    const FitJob &j = jobs[blockIdx.x];
    fit_finish_body(j.R, j.lambda, j.GA, j.GB, j.GC, j.part, j.nblk, j.normsq, j.fit, sh);
}

template <bool SMEM>
__global__ __launch_bounds__(kBlock) void k_als_lambda(
    int R, int mode, const double *__restrict__ Hinv_g, const double *__restrict__ MtM_g,
    double *__restrict__ Gn, double *__restrict__ W, double *__restrict__ lambda_out,
    const double *__restrict__ GA, const double *__restrict__ GB, double normsq,
    double *__restrict__ fit_out, double *__restrict__ scratch) {
    extern __shared__ double dyn[];
    als_lambda_body<SMEM>(R, mode, Hinv_g, MtM_g, Gn, W, lambda_out, GA, GB, normsq, fit_out,
                          scratch, dyn);
}

template <bool SMEM>
__global__ __launch_bounds__(kBlock) void k_als_lambda_group(const LambdaJob *__restrict__ jobs) {
    extern __shared__ double dyn[];
    const LambdaJob &j = jobs[blockIdx.x];
    als_lambda_body<SMEM>(j.R, j.mode, j.Hinv, j.MtM, j.Gn, j.W, j.lambda, j.GA, j.GB, j.normsq,
                          j.fit, j.scratch, dyn);
}

// ---------------------------------------------------------------------------
// Row maps over tiles of TR = kTileElems / R consecutive rows (one contiguous
// block of memory): the tile is loaded with coalesced loads into LDS (row
// stride R + 1, conflict-free column reads), each thread computes CT = 16
// columns of one row with the R x R matrix broadcast from LDS (all lanes of a
// wave work on the same columns), and the result tile is written back with
// coalesced stores.  Instantiated for R in {4, 8, 12, 16, 32, 48}.
// ---------------------------------------------------------------------------
constexpr int kTileElems = 4096;
constexpr int kCT = 16;  // columns per thread

__host__ __device__ constexpr int tile_rows(int R) { return kTileElems / R < kBlock ? kTileElems / R : kBlock; }

template <typename T>
__device__ __forceinline__ float ldf(const T *p, int64_t i);
template <>
__device__ __forceinline__ float ldf<float>(const float *p, int64_t i) { return p[i]; }
template <>
__device__ __forceinline__ float ldf<uint16_t>(const uint16_t *p, int64_t i) {
    return __uint_as_float((uint32_t)p[i] << 16);
}

// F[row, s] = sum_k M[row, k] W[k, s]   (R is a compile-time constant)
template <typename Tout, int R>
__device__ __forceinline__ void rowmap_t_body(const float *__restrict__ M, int64_t rows,
                                              const double *__restrict__ W, Tout *__restrict__ F,
                                              double *dyn, uint32_t b, uint32_t nb) {
    double *sW = dyn;                                  // R * R
    float *sM = reinterpret_cast<float *>(sW + R * R);  // TR * (R + 1)
    constexpr int TR = tile_rows(R), RS = R + 1;
    float *sO = sM + TR * RS;                          // TR * (R + 1)
    for (int e = threadIdx.x; e < R * R; e += kBlock) sW[e] = W[e];
    constexpr int tpr = kBlock / TR;                   // threads per row
    const int rr = threadIdx.x % TR, part = threadIdx.x / TR;
    const int c0 = part * kCT;
    const bool active = part < tpr && c0 < R;
    const int64_t ntile = (rows + TR - 1) / TR;
    for (int64_t tile = b; tile < ntile; tile += nb) {
        const int64_t r0 = tile * TR;
        const int nr = (int)((rows - r0) < TR ? (rows - r0) : TR);
        __syncthreads();
        for (int e = threadIdx.x; e < nr * R; e += kBlock) sM[(e / R) * RS + e % R] = M[r0 * R + e];
        __syncthreads();
        if (active && rr < nr) {
            double acc[kCT];
#pragma unroll
            for (int s = 0; s < kCT; ++s) acc[s] = 0.0;
            const float *m = sM + rr * RS;
#pragma unroll 4
            for (int k = 0; k < R; ++k) {
                const double mk = m[k];
                const double *w = sW + k * R + c0;
#pragma unroll
                for (int s = 0; s < kCT; ++s)
                    if (c0 + s < R) acc[s] = fma(mk, w[s], acc[s]);
            }
#pragma unroll
            for (int s = 0; s < kCT; ++s)
                if (c0 + s < R) sO[rr * RS + c0 + s] = (float)acc[s];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < nr * R; e += kBlock)
            st_out<Tout>(F, r0 * R + e, (double)sO[(e / R) * RS + e % R]);
    }
}

template <typename Tout, int R>
__global__ __launch_bounds__(kBlock) void k_rowmap_t(const float *__restrict__ M, int64_t rows,
                                                     const double *__restrict__ W,
                                                     Tout *__restrict__ F) {
    extern __shared__ double dyn[];
    rowmap_t_body<Tout, R>(M, rows, W, F, dyn, blockIdx.x, gridDim.x);
}

template <typename Tout, int R>
__global__ __launch_bounds__(kBlock) void k_rowmap_t_group(const RowmapJob *__restrict__ jobs,
                                                           const uint2 *__restrict__ vb) {
    extern __shared__ double dyn[];
    const uint2 v = vb[blockIdx.x];
    const RowmapJob &j = jobs[v.x];
    rowmap_t_body<Tout, R>(j.M, j.rows, j.W, (Tout *)j.F, dyn, v.y, j.nblk);
}

// G[row, s] = -G[row, s] + sum_k F[row, k] H[k, s]  (G holds the MTTKRP);
// partial[block] = sum over the block's rows of <F[row,:], M[row,:]>.
template <typename T, int R>
__global__ __launch_bounds__(kBlock) void k_gd_rows_t(float *__restrict__ G,
                                                      const T *__restrict__ F, int64_t rows,
                                                      const double *__restrict__ H,
                                                      double *__restrict__ partial) {
    extern __shared__ double dyn[];
    __shared__ double sh[kBlock];
    double *sH = dyn;
    float *sF = reinterpret_cast<float *>(sH + R * R);
    constexpr int TR = tile_rows(R), RS = R + 1;
    float *sM = sF + TR * RS;
    for (int e = threadIdx.x; e < R * R; e += kBlock) sH[e] = H[e];
    constexpr int tpr = kBlock / TR;
    const int rr = threadIdx.x % TR, part = threadIdx.x / TR;
    const int c0 = part * kCT;
    const bool active = part < tpr && c0 < R;
    const int64_t ntile = (rows + TR - 1) / TR;
    double inner = 0.0;
    for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        const int64_t r0 = tile * TR;
        const int nr = (int)((rows - r0) < TR ? (rows - r0) : TR);
        __syncthreads();
        for (int e = threadIdx.x; e < nr * R; e += kBlock) {
            const int o = (e / R) * RS + e % R;
            sF[o] = ldf<T>(F, r0 * R + e);
            sM[o] = G[r0 * R + e];
        }
        __syncthreads();
        double acc[kCT];
        if (active && rr < nr) {
#pragma unroll
            for (int s = 0; s < kCT; ++s) acc[s] = 0.0;
            const float *f = sF + rr * RS;
#pragma unroll 4
            for (int k = 0; k < R; ++k) {
                const double fk = f[k];
                const double *h = sH + k * R + c0;
#pragma unroll
                for (int s = 0; s < kCT; ++s)
                    if (c0 + s < R) acc[s] = fma(fk, h[s], acc[s]);
            }
        }
        __syncthreads();  // every thread has read its F row: sF can take the output
        if (active && rr < nr) {
            const float *mrow = sM + rr * RS;
#pragma unroll
            for (int s = 0; s < kCT; ++s) {
                if (c0 + s < R) {
                    const double m = mrow[c0 + s];
                    inner = fma((double)sF[rr * RS + c0 + s], m, inner);
                }
            }
        }
        __syncthreads();
        if (active && rr < nr) {
            const float *mrow = sM + rr * RS;
#pragma unroll
            for (int s = 0; s < kCT; ++s)
                if (c0 + s < R) sF[rr * RS + c0 + s] = (float)(acc[s] - (double)mrow[c0 + s]);
        }
        __syncthreads();
        for (int e = threadIdx.x; e < nr * R; e += kBlock) G[r0 * R + e] = sF[(e / R) * RS + e % R];
    }
    const double tot = block_sum(inner, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

size_t tile_lds_bytes(int R) {
    return sizeof(double) * (size_t)R * R + 2 * sizeof(float) * (size_t)tile_rows(R) * (R + 1);
}

// Generic versions for any R (up to 256): rows staged in LDS, the matrix in
// LDS when it fits.
constexpr int kLdsMatMaxR = 64;

template <typename Tout>
__global__ __launch_bounds__(kBlock) void k_rowmap_g(const float *__restrict__ M, int64_t rows,
                                                     int R, const double *__restrict__ W,
                                                     Tout *__restrict__ F) {
    __shared__ double sW[kLdsMatMaxR * kLdsMatMaxR];
    __shared__ float sM[kBlock * 4];
    const bool wlds = R <= kLdsMatMaxR;
    if (wlds)
        for (int e = threadIdx.x; e < R * R; e += kBlock) sW[e] = W[e];
    const int rpp = (kBlock * 4) / R > 0 ? (kBlock * 4) / R : 1;  // rows per pass staged
    const int64_t npass = (rows + rpp - 1) / rpp;
    for (int64_t pass = blockIdx.x; pass < npass; pass += gridDim.x) {
        const int64_t r0 = pass * rpp;
        const int nr = (int)((rows - r0) < rpp ? (rows - r0) : rpp);
        __syncthreads();
        for (int e = threadIdx.x; e < nr * R; e += kBlock) sM[e] = M[r0 * R + e];
        __syncthreads();
        for (int e = threadIdx.x; e < nr * R; e += kBlock) {
            const int rr = e / R, s = e % R;
            double acc = 0.0;
            const float *m = sM + rr * R;
            if (wlds) {
                for (int k = 0; k < R; ++k) acc = fma((double)m[k], sW[k * R + s], acc);
            } else {
                for (int k = 0; k < R; ++k) acc = fma((double)m[k], W[k * R + s], acc);
            }
            st_out<Tout>(F, r0 * R + e, acc);
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_gd_rows_g(float *__restrict__ G, const T *__restrict__ F,
                                                      int64_t rows, int R,
                                                      const double *__restrict__ H,
                                                      double *__restrict__ partial) {
    __shared__ double sH[kLdsMatMaxR * kLdsMatMaxR];
    __shared__ double sF[kBlock * 2];
    __shared__ double sh[kBlock];
    const bool hlds = R <= kLdsMatMaxR;
    if (hlds)
        for (int e = threadIdx.x; e < R * R; e += kBlock) sH[e] = H[e];
    const int rpp = (kBlock * 2) / R > 0 ? (kBlock * 2) / R : 1;
    const int64_t npass = (rows + rpp - 1) / rpp;
    double inner = 0.0;
    for (int64_t pass = blockIdx.x; pass < npass; pass += gridDim.x) {
        const int64_t r0 = pass * rpp;
        const int nr = (int)((rows - r0) < rpp ? (rows - r0) : rpp);
        __syncthreads();
        for (int e = threadIdx.x; e < nr * R; e += kBlock) sF[e] = ld<T>(F, r0 * R + e);
        __syncthreads();
        for (int e = threadIdx.x; e < nr * R; e += kBlock) {
            const int rr = e / R, s = e % R;
            const double *f = sF + rr * R;
            double acc = 0.0;
            if (hlds) {
                for (int k = 0; k < R; ++k) acc = fma(f[k], sH[k * R + s], acc);
            } else {
                for (int k = 0; k < R; ++k) acc = fma(f[k], H[k * R + s], acc);
            }
            const double m = (double)G[r0 * R + e];
            inner = fma(f[s], m, inner);
            G[r0 * R + e] = (float)(acc - m);
        }
    }
    const double tot = block_sum(inner, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_gd_f(int R, const double *__restrict__ GA,
                                                 const double *__restrict__ GB,
                                                 const double *__restrict__ GC,
                                                 const double *__restrict__ partial, int npartial,
                                                 double normsq, double reg, double *__restrict__ f) {
    __shared__ double sh[kBlock];
    double in = 0.0;
    for (int b = threadIdx.x; b < npartial; b += kBlock) in += partial[b];
    double xh = 0.0, tr = 0.0;
    for (int e = threadIdx.x; e < R * R; e += kBlock) {
        xh += GA[e] * GB[e] * GC[e];
        if (e / R == e % R) tr += GA[e] + GB[e] + GC[e];
    }
    in = block_sum(in, sh);
    xh = block_sum(xh, sh);
    tr = block_sum(tr, sh);
    if (threadIdx.x == 0) *f = 0.5 * (normsq - 2.0 * in + xh) + 0.5 * reg * tr;
}

// ---- GD step: trial factors and the squared gradient norm ----------------
// out = F - alpha * G, formed in FP64 from the stored factor and the FP32
// gradient, stored in the factor dtype (BF16: FP32 then nearest-even BF16)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_trial_factor(const T *__restrict__ F,
                                                         const float *__restrict__ G, double alpha,
                                                         T *__restrict__ out, int64_t n) {
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kBlock)
        st_out<T>(out, e, ld<T>(F, e) - alpha * (double)G[e]);
}

// per-block partial sums of x^2 in FP64 (grid-stride, fixed order)
__global__ __launch_bounds__(kBlock) void k_sumsq_f32(const float *__restrict__ x, int64_t n,
                                                      double *__restrict__ part) {
    __shared__ double sh[kBlock];
    double acc = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kBlock) {
        const double v = (double)x[e];
        acc += v * v;
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ __launch_bounds__(kBlock) void k_sum_parts(const double *__restrict__ part, int n,
                                                      double *__restrict__ out) {
    __shared__ double sh[kBlock];
    double acc = 0.0;
    for (int b = threadIdx.x; b < n; b += kBlock) acc += part[b];
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) *out = acc;
}

// ---- joint matrix completion + tensor factorization ----------------------
// One ALS row of the joint model per wave (R <= 32).  For the stored
// entries of the row in a ratings stream (headers name the mid row,
// nonzeros the leaf row and the rating y; the entry's vector is
// v = F_mid[mid] * F_leaf[leaf], the other factor's row when the third
// factor is a row of ones) the wave forms in FP64
//   S = sum v^T v + mu H + lam I,   rhs = sum y v + mu M[row]
// solves S x = rhs by Cholesky and writes out[row] = x in the factor dtype.
// Register layout: lane (h, r) = (lane / 32, lane % 32) keeps
// S[r][2k + h], k < 16, so both half-waves work on the row; entries, rows
// and columns beyond R are zero.  Entries are taken 32 at a time (two lanes
// load each entry's vector into LDS, all loads of a batch in flight
// together), then the wave adds the batch's outer products in entry order.
// Rows longer than kJointSeg entries are split into segments whose partial
// (S, rhs) go to `part` and are summed in segment order by k_joint_heavy.
// A row whose S fails the positive-definiteness test is written as zeros and
// raises *flag.
constexpr int kJointRM = 32;            // largest rank
constexpr int kJointRP = kJointRM + 1;  // padded LDS row
constexpr int kJointK = kJointRM / 2;   // columns of S per lane
constexpr int kJointB = 32;             // entries per batch

// lane `src`'s v (src uniform) in every lane
__device__ __forceinline__ double lane_bcast(double v, int src) {
    const long long x = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(x & 0xffffffffll), src);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(x >> 32), src);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// lane (h, r): p[k] = (mu H + lam I)[r][2k + h] (zero outside R x R)
__device__ __forceinline__ void joint_shift(const double *__restrict__ H, int R, double mu,
                                            double lam, double (&p)[kJointK]) {
    const int h = threadIdx.x >> 5, r = threadIdx.x & 31;
#pragma unroll
    for (int k = 0; k < kJointK; ++k) {
        const int q = 2 * k + h;
        p[k] = (r < R && q < R) ? mu * H[r * R + q] + (q == r ? lam : 0.0) : 0.0;
    }
}

// One batch [b, min(b + 32, e1)) of a ratings stream: the nonzeros'
// vectors go, compacted in stream order, to rows 0 .. n-1 of V (columns
// beyond R zero) and their ratings to Yb; returns n.  cur_mid is the mid row
// of the fiber open at b and comes back as the one open at the batch's end.
template <typename T>
__device__ int joint_load_batch(const uint2 *__restrict__ st, uint32_t b, uint32_t e1,
                                const T *__restrict__ Fmid, const T *__restrict__ Fleaf, int R,
                                uint32_t &cur_mid, double *V, double *Yb) {
    const int h = threadIdx.x >> 5, t = threadIdx.x & 31;
    // entry t of the batch in lanes t and t + 32
    const uint32_t e = b + (uint32_t)t;
    const bool in = e < e1;
    const uint2 w = in ? st[e] : make_uint2(0u, 0u);
    const bool hdr = in && (w.x & kHdrBit);
    const bool nz = in && !(w.x & kHdrBit);
    const uint64_t hm = __ballot(hdr) & 0xffffffffull;
    const uint64_t nm = __ballot(nz) & 0xffffffffull;
    const uint64_t upto = hm & ((2ull << t) - 1ull);
    const uint32_t midx = w.x & kIdxMask;
    const uint32_t lastm = hm ? (uint32_t)__shfl((int)midx, 63 - __clzll((long long)hm)) : 0u;
    const uint32_t srcm = upto ? (uint32_t)__shfl((int)midx, 63 - __clzll((long long)upto)) : 0u;
    const uint32_t my_mid = upto ? srcm : cur_mid;
    if (hm) cur_mid = lastm;
    if (nz) {
        const int slot = __popcll(nm & ((1ull << t) - 1ull));
        const T *pm = Fmid + (int64_t)my_mid * R;
        const T *pl = Fleaf + (int64_t)w.x * R;
#pragma unroll
        for (int k = 0; k < kJointK; ++k) {
            const int q = 2 * k + h;
            V[slot * kJointRP + q] = q < R ? ld<T>(pm, q) * ld<T>(pl, q) : 0.0;
        }
        if (h == 0) Yb[slot] = (double)__uint_as_float(w.y);
    }
    __syncthreads();
    return __popcll(nm);
}

// c[k] += sum_u v_u[r] v_u[2k + h], rhs += sum_u y_u v_u[r] over the n
// loaded entries, in order
__device__ __forceinline__ void joint_add_batch(int n, double (&c)[kJointK], double &rhs,
                                                const double *V, const double *Yb) {
    const int h = threadIdx.x >> 5, t = threadIdx.x & 31;
    for (int u = 0; u < n; ++u) {
        const double vr = V[u * kJointRP + t];  // v[r]: zero for r >= R
        rhs = fma(Yb[u], vr, rhs);
#pragma unroll
        for (int k = 0; k < kJointK; ++k) c[k] = fma(V[u * kJointRP + 2 * k + h], vr, c[k]);
    }
    __syncthreads();
}

// c[k] += sum over the entries [e0, e1) of v[r] v[2k + h]; rhs += sum y v[r]
template <typename T, bool kSegment>
__device__ void joint_accumulate(const uint2 *__restrict__ st, uint32_t e0, uint32_t e1,
                                 const T *__restrict__ Fmid, const T *__restrict__ Fleaf, int R,
                                 double (&c)[kJointK], double &rhs, double *V, double *Yb) {
    const int l = threadIdx.x;
    // a segment may start inside a fiber: the fiber's header is at most one
    // fiber (<= kFiberCap nonzeros) before e0, and the row's first entry is a
    // header (a whole row starts with one)
    uint32_t cur_mid = 0;
    if (kSegment && !(st[e0].x & kHdrBit)) {
        for (uint32_t back = 0; back < e0; back += 64) {
            const uint32_t e = e0 - 1 - back - (uint32_t)l;  // e0 - 1 - back - l >= row start here
            const bool in = back + (uint32_t)l < e0;
            const uint2 w = in ? st[e] : make_uint2(0u, 0u);
            const uint64_t hb = __ballot(in && (w.x & kHdrBit));
            if (hb) {
                const int src = __ffsll((unsigned long long)hb) - 1;  // the nearest header
                cur_mid = (uint32_t)__shfl((int)(w.x & kIdxMask), src);
                break;
            }
        }
    }
    for (uint32_t b = e0; b < e1; b += kJointB) {
        const int n = joint_load_batch<T>(st, b, e1, Fmid, Fleaf, R, cur_mid, V, Yb);
        joint_add_batch(n, c, rhs, V, Yb);
    }
}

// A row of at most kJointWood entries (vectors v_e in rows of V, ratings in
// Yb) solved without factorizing its own S = P + V^T V, from P^-1 (the same
// for every row of the mode) by the Sherman-Morrison-Woodbury identity:
//   b = sum_e y_e v_e + mu m,  z = P^-1 b,  u_e = P^-1 v_e,
//   K = I + [v_e . u_f],  t = [v_e . z],  K w = t,  x = z - sum_e w_e u_e.
// P^-1 = ws * Pinv (R x R, row-major), or ws * I when Pinv is null.  K is
// symmetric positive definite with eigenvalues >= 1 and is solved by
// Gauss-Jordan without pivoting, lane (e, f) = e * 8 + f holding K[e][f]
// and lane (e, n) holding t[e].  U (kJointRM rows of kJointRP doubles, apart
// from V's first n rows) holds u_e and z; Bb (32 doubles) carries b.
constexpr int kJointWood = 7;

// (not inlined: inside the rows kernel's loop it would cost a wave per SIMD
// of registers)
template <typename T>
__device__ __noinline__ void joint_woodbury(int n, const double *V, const double *Yb, double mu, double m,
                               const double *__restrict__ Pinv, double ws, int R, int64_t row,
                               T *__restrict__ out, double *U, double *Bb) {
    const int l = threadIdx.x, h = l >> 5, r = l & 31;
    double wr[kJointK];  // P^-1[r][2k + h]
#pragma unroll
    for (int k = 0; k < kJointK; ++k) {
        const int q = 2 * k + h;
        wr[k] = (r < R && q < R) ? (Pinv ? ws * Pinv[r * R + q] : (q == r ? ws : 0.0)) : 0.0;
    }
    double b = 0.0;
    for (int e = 0; e < n; ++e) b = fma(Yb[e], V[e * kJointRP + r], b);
    b = fma(mu, m, b);
    if (h == 0) Bb[r] = b;
    __syncthreads();
    double zp = 0.0;
#pragma unroll
    for (int k = 0; k < kJointK; ++k) zp = fma(wr[k], Bb[2 * k + h], zp);
    const double z = zp + __shfl_xor(zp, 32, 64);  // the halves' sums, equal in both
    for (int e = 0; e < n; ++e) {
        double up = 0.0;
#pragma unroll
        for (int k = 0; k < kJointK; ++k) up = fma(wr[k], V[e * kJointRP + 2 * k + h], up);
        const double u = up + __shfl_xor(up, 32, 64);
        if (h == 0) U[e * kJointRP + r] = u;
    }
    if (h == 0) U[n * kJointRP + r] = z;
    __syncthreads();
    // G[e][f] = a_e . v_f for e <= n (a_e = u_e, a_n = z) and f < n
    const int ge = l >> 3, gf = l & 7;
    double g = 0.0;
    if (ge <= n && gf < n) {
#pragma unroll 4
        for (int q = 0; q < kJointRM; ++q) g = fma(U[ge * kJointRP + q], V[gf * kJointRP + q], g);
    }
    const double tv = __shfl(g, n * 8 + ge, 64);  // t[ge] = z . v_ge
    double a = 0.0;
    if (ge < n && gf < n) a = g + (ge == gf ? 1.0 : 0.0);
    if (ge < n && gf == n) a = tv;
    for (int j = 0; j < n; ++j) {
        const double inv = 1.0 / lane_bcast(a, j * 9);  // K's pivot at step j
        const double rowj = __shfl(a, j * 8 + gf, 64);
        const double colj = __shfl(a, ge * 8 + j, 64);
        a = ge == j ? rowj * inv : fma(-colj * inv, rowj, a);
    }
    double x = z;
    for (int e = 0; e < n; ++e) x = fma(-lane_bcast(a, e * 8 + n), U[e * kJointRP + r], x);
    if (h == 0 && r < R) st_out<T>(out, row * R + r, x);
    __syncthreads();  // U, V and Bb are free again
}

// S = c + p (p = mu H + lam I in the same layout); b = rhs (lane (h, r)
// holds rhs[r]).  Cholesky S = L L^T with
// the pivot test d_j > R eps max diag(S), forward substitution folded into
// the factorization, then L^T x = y after one transpose of L through LDS;
// out[row] = x.  Lc (2 x 32 doubles) carries the current column of L,
// Tl (32 x kJointRP doubles) the transpose.
template <typename T>
__device__ void joint_solve_store(double (&c)[kJointK], double b, const double (&p)[kJointK],
                                  int64_t row, int R, T *__restrict__ out,
                                  int *__restrict__ flag, double *Lc, double *Tl) {
    const int l = threadIdx.x, h = l >> 5, r = l & 31;
    double dl = 0.0;
#pragma unroll
    for (int k = 0; k < kJointK; ++k) {
        const int q = 2 * k + h;
        c[k] += p[k];
        if (q == r) dl = c[k];
    }
    double dm = dl;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) dm = fmax(dm, __shfl_xor(dm, o, 64));
    const double tol = (double)R * DBL_EPSILON * dm;
    bool ok = dm > 0.0;
    double myinv = 0.0;  // 1 / L[r][r]
    // fully unrolled (no early exit): every index into c is a constant
#pragma unroll
    for (int j = 0; j < kJointRM; ++j) {
        const int jh = j & 1, jk = j >> 1;
        const double d = lane_bcast(c[jk], jh * 32 + j);  // the Schur-complement pivot
        if (j < R && ok) ok = d > tol;
        if (j < R && ok) {
            const double inv = rsqrt(d);
            double *lc = Lc + jh * 32;  // two buffers: no barrier before the next write
            if (h == jh) lc[r] = r > j ? c[jk] * inv : 0.0;
            const double yj = lane_bcast(b, j) * inv;
            if (r == j) myinv = inv;
            __syncthreads();
            const double lr = lc[r];  // L[r][j], zero for r <= j
            if (h == jh && r > j) c[jk] = lr;
            b = r == j ? yj : fma(-lr, yj, b);
            double lk[kJointK];  // all reads of the column in flight together
#pragma unroll
            for (int k = jk; k < kJointK; ++k) lk[k] = lc[2 * k + h];
#pragma unroll
            for (int k = jk; k < kJointK; ++k) c[k] = fma(-lr, lk[k], c[k]);
        }
    }
    if (ok) {
        // L^T x = y: lane (h, r) keeps lt[k] = L[2k + h][r] and in acc the
        // sum of L[j][r] x_j over the solved j of its parity h, so
        // x_j = (y_j - acc(0, j) - acc(1, j)) / L[j][j]
#pragma unroll
        for (int k = 0; k < kJointK; ++k) Tl[r * kJointRP + 2 * k + h] = c[k];
        __syncthreads();
        double lt[kJointK];
#pragma unroll
        for (int k = 0; k < kJointK; ++k) lt[k] = Tl[(2 * k + h) * kJointRP + r];
        double acc = 0.0, x = 0.0;
#pragma unroll
        for (int j = kJointRM - 1; j >= 0; --j) {
            if (j < R) {
                const double xj = (lane_bcast(b - acc, j) - lane_bcast(acc, 32 + j)) *
                                  lane_bcast(myinv, j);
                if (r == j) x = xj;
                if (h == (j & 1) && r < j) acc = fma(lt[j >> 1], xj, acc);
            }
        }
        b = x;
    }
    __syncthreads();  // Tl and Lc are free again
    if (h == 0 && r < R) st_out<T>(out, row * R + r, ok ? b : 0.0);
    if (!ok && l == 0) atomicOr(flag, 1);
}

// every row of at most kJointSeg entries: accumulate, solve, store
// (persistent grid: each workgroup forms mu H + lam I once and walks rows)
// Rows whose stream range fits one batch and holds at most kJointWood
// entries take joint_woodbury when P^-1 is valid (Pinv null, or its solve
// reported success in *pflag == 0).
template <typename T>
__global__ __launch_bounds__(64) void k_joint_rows(const uint2 *__restrict__ st,
                                                   const uint2 *__restrict__ range, int64_t nrows,
                                                   const T *__restrict__ Fmid,
                                                   const T *__restrict__ Fleaf, int R,
                                                   const float *__restrict__ M,
                                                   const double *__restrict__ H, double mu,
                                                   double lam, const double *__restrict__ Pinv,
                                                   double ws, const int *__restrict__ pflag,
                                                   T *__restrict__ out, int *__restrict__ flag) {
    __shared__ double V[kJointB * kJointRP], Yb[kJointB], Lc[2 * 32];
    const int r = threadIdx.x & 31;
    double p[kJointK];
    joint_shift(H, R, mu, lam, p);
    const bool wood = !Pinv || *pflag == 0;
    uint2 next = blockIdx.x < nrows ? range[blockIdx.x] : make_uint2(0u, 0u);
    for (int64_t row = blockIdx.x; row < nrows; row += gridDim.x) {
        const uint2 rg = next;  // the next row's range is read while this one is solved
        if (row + gridDim.x < nrows) next = range[row + gridDim.x];
        if (rg.y - rg.x > (uint32_t)kJointSeg) continue;  // a heavy row: segments below
        const double m = (M && r < R) ? (double)M[row * R + r] : 0.0;
        double c[kJointK];
#pragma unroll
        for (int k = 0; k < kJointK; ++k) c[k] = 0.0;
        double rhs = 0.0;
        if (wood && rg.y - rg.x <= (uint32_t)kJointB) {
            uint32_t cur_mid = 0;
            const int n =
                rg.y > rg.x ? joint_load_batch<T>(st, rg.x, rg.y, Fmid, Fleaf, R, cur_mid, V, Yb)
                            : 0;
            if (n <= kJointWood) {
                joint_woodbury<T>(n, V, Yb, mu, m, Pinv, ws, R, row, out,
                                  V + 16 * kJointRP, Lc);
                continue;
            }
            joint_add_batch(n, c, rhs, V, Yb);
        } else if (rg.y > rg.x) {
            joint_accumulate<T, false>(st, rg.x, rg.y, Fmid, Fleaf, R, c, rhs, V, Yb);
        }
        if (M) rhs = fma(mu, m, rhs);
        joint_solve_store<T>(c, rhs, p, row, R, out, flag, Lc, V);
    }
}

// one segment of a heavy row: partial S (R x R, row-major) and rhs (R)
template <typename T>
__global__ __launch_bounds__(64) void k_joint_segments(const uint2 *__restrict__ st,
                                                       const uint2 *__restrict__ seg,
                                                       int64_t nseg, const T *__restrict__ Fmid,
                                                       const T *__restrict__ Fleaf, int R,
                                                       double *__restrict__ part) {
    __shared__ double V[kJointB * kJointRP], Yb[kJointB];
    const int h = threadIdx.x >> 5, r = threadIdx.x & 31;
    for (int64_t q = blockIdx.x; q < nseg; q += gridDim.x) {
        const uint2 sg = seg[q];
        double c[kJointK];
#pragma unroll
        for (int k = 0; k < kJointK; ++k) c[k] = 0.0;
        double rhs = 0.0;
        joint_accumulate<T, true>(st, sg.x, sg.y, Fmid, Fleaf, R, c, rhs, V, Yb);
        double *P = part + q * (int64_t)(R * R + R);
        if (r < R) {
#pragma unroll
            for (int k = 0; k < kJointK; ++k)
                if (2 * k + h < R) P[r * R + 2 * k + h] = c[k];
            if (h == 0) P[R * R + r] = rhs;
        }
    }
}

// a heavy row: the sum of its segments' partials in segment order, solved
template <typename T>
__global__ __launch_bounds__(64) void k_joint_heavy(const uint4 *__restrict__ heavy,
                                                    int64_t nheavy, int R,
                                                    const double *__restrict__ part,
                                                    const float *__restrict__ M,
                                                    const double *__restrict__ H, double mu,
                                                    double lam, T *__restrict__ out,
                                                    int *__restrict__ flag) {
    __shared__ double Tl[kJointRM * kJointRP], Lc[2 * 32];
    const int h = threadIdx.x >> 5, r = threadIdx.x & 31;
    double p[kJointK];
    joint_shift(H, R, mu, lam, p);
    for (int64_t hi = blockIdx.x; hi < nheavy; hi += gridDim.x) {
        const uint4 hv = heavy[hi];  // (row, first segment, segments, 0)
        double c[kJointK];
#pragma unroll
        for (int k = 0; k < kJointK; ++k) c[k] = 0.0;
        double rhs = 0.0;
        if (r < R) {
            for (uint32_t q = hv.y; q < hv.y + hv.z; ++q) {
                const double *P = part + (int64_t)q * (R * R + R);
#pragma unroll
                for (int k = 0; k < kJointK; ++k)
                    if (2 * k + h < R) c[k] += P[r * R + 2 * k + h];
                rhs += P[R * R + r];
            }
        }
        if (M && r < R) rhs = fma(mu, (double)M[(int64_t)hv.x * R + r], rhs);
        joint_solve_store<T>(c, rhs, p, (int64_t)hv.x, R, out, flag, Lc, Tl);
    }
}

// G = mu G + lam F - RY (RY may be null): the joint gradient from the
// tensor part -M + F H, the ridge term and the ratings part
template <typename T>
__global__ __launch_bounds__(kBlock) void k_joint_combine(float *__restrict__ G,
                                                          const T *__restrict__ F,
                                                          const float *__restrict__ RY, double mu,
                                                          double lam, int64_t n) {
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kBlock) {
        double g = mu * (double)G[e] + lam * ld<T>(F, e);
        if (RY) g -= (double)RY[e];
        G[e] = (float)g;
    }
}

// per-block partial sums of F[e] * X[e] in FP64 (grid-stride, fixed order)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dot_parts(const T *__restrict__ F,
                                                      const float *__restrict__ X, int64_t n,
                                                      double *__restrict__ part) {
    __shared__ double sh[kBlock];
    double acc = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kBlock)
        acc = fma(ld<T>(F, e), (double)X[e], acc);
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// f = mu f_tensor + lam/2 (tr G_A + tr G_B + tr G_C)
//     + 1/2 (||Y||^2 - <A, Y B> - <A, residual(Y) B>)
// (the ratings term: sum r^2 = sum r y - sum r (a.b) = ||Y||^2 - <A,YB> - <A,RB>)
__global__ __launch_bounds__(kBlock) void k_joint_f(const double *__restrict__ ft,
                                                    const double *__restrict__ GA,
                                                    const double *__restrict__ GB,
                                                    const double *__restrict__ GC, int R,
                                                    const double *__restrict__ part, int npart,
                                                    double normsq_y, double mu, double lam,
                                                    double *__restrict__ f) {
    __shared__ double sh[kBlock];
    double in = 0.0, tr = 0.0;
    for (int b = threadIdx.x; b < npart; b += kBlock) in += part[b];
    for (int r = threadIdx.x; r < R; r += kBlock) tr += GA[r * R + r] + GB[r * R + r] + GC[r * R + r];
    in = block_sum(in, sh);
    tr = block_sum(tr, sh);
    if (threadIdx.x == 0) *f = mu * ft[0] + 0.5 * lam * tr + 0.5 * (normsq_y - in);
}

// 16-byte row loads are allowed when every row start is 16-byte aligned
int vec_rows(const void *p, int R, int elem) {
    return ((uintptr_t)p % 16 == 0) && (((size_t)R * elem) % 16 == 0);
}

// ---------------------------------------------------------------------------
// Row maps on the matrix cores, R = 16 * NCT (16, 32, 48, 64).
//
// A wave takes 16 rows X[r0 .. r0+16) at a time and forms out^T = W^T X^T with
// FP64 MFMA 16x16x4 steps: the R x R matrix is the A operand and stays in
// registers for the whole kernel (4 * NCT^2 doubles per lane), the rows are
// the B operand.  Two index permutations make every lane's memory accesses
// 4 consecutive elements wide:
//  * contraction index: at step t, lane group g = lane / 16 contributes
//    k = 16 * (t / 4) + 4 * g + t % 4, so a lane reads columns
//    16 * c + 4 * g .. + 4 of its row for c = 0 .. NCT-1;
//  * output index: MFMA output row m of column tile c is column
//    16 * c + 4 * (m % 4) + m / 4, so the 4 accumulator entries of a lane are
//    columns 16 * c + 4 * g .. + 4 of row r0 + lane % 16 -- the same columns
//    it read.
// Accumulation is FP64; the next tile's rows are loaded before the current
// tile's MFMAs.
// ---------------------------------------------------------------------------
// Raw 4-element runs (kept undecoded while in flight: half the registers of
// doubles for FP32, a quarter for BF16).
template <typename T>
struct Run4;
template <>
struct Run4<float> {
    float4 v;
    __device__ __forceinline__ void load(const float *p) { v = *reinterpret_cast<const float4 *>(p); }
    __device__ __forceinline__ void zero() { v = make_float4(0.f, 0.f, 0.f, 0.f); }
    __device__ __forceinline__ double operator[](int i) const {
        return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
    }
};
template <>
struct Run4<uint16_t> {
    uint2 v;
    __device__ __forceinline__ void load(const uint16_t *p) { v = *reinterpret_cast<const uint2 *>(p); }
    __device__ __forceinline__ void zero() { v = make_uint2(0u, 0u); }
    __device__ __forceinline__ double operator[](int i) const {
        const uint32_t w = i < 2 ? v.x : v.y;
        return __uint_as_float((i % 2 == 0) ? (w << 16) : (w & 0xFFFF0000u));
    }
};
__device__ __forceinline__ void store4d(float *p, const double4v &a) {
    *reinterpret_cast<float4 *>(p) = make_float4((float)a[0], (float)a[1], (float)a[2], (float)a[3]);
}
__device__ __forceinline__ void store4d(uint16_t *p, const double4v &a) {
    uint2 w;
    w.x = (uint32_t)f32_to_bf16((float)a[0]) | ((uint32_t)f32_to_bf16((float)a[1]) << 16);
    w.y = (uint32_t)f32_to_bf16((float)a[2]) | ((uint32_t)f32_to_bf16((float)a[3]) << 16);
    *reinterpret_cast<uint2 *>(p) = w;
}

// wa[c][t] = W[k(t)][16 c + column of MFMA row lane % 16]
template <int NCT>
__device__ __forceinline__ void load_rmat(const double *__restrict__ W, int lane,
                                          double (&wa)[NCT][4 * NCT]) {
    constexpr int R = 16 * NCT;
    const int g = lane / 16, m = lane % 16;
    const int col = 4 * (m % 4) + m / 4;
#pragma unroll
    for (int c = 0; c < NCT; ++c)
#pragma unroll
        for (int t = 0; t < 4 * NCT; ++t) {
            const int k = 16 * (t / 4) + 4 * g + t % 4;
            wa[c][t] = W[k * R + 16 * c + col];
        }
}

// the 4 * NCT entries of row `row` that this lane reads (zero past the last row)
template <int NCT, typename T>
__device__ __forceinline__ void load_rowrun(const T *__restrict__ X, int64_t row, int64_t rows,
                                            int g, Run4<T> (&v)[NCT]) {
    constexpr int R = 16 * NCT;
    if (row < rows) {
#pragma unroll
        for (int c = 0; c < NCT; ++c) v[c].load(X + row * R + 16 * c + 4 * g);
    } else {
#pragma unroll
        for (int c = 0; c < NCT; ++c) v[c].zero();
    }
}

// F[row, s] = sum_k M[row, k] W[k, s]
template <typename Tout, int NCT>
__device__ __forceinline__ void rowmap_mfma_body(const float *__restrict__ M, int64_t rows,
                                                 const double *__restrict__ W,
                                                 Tout *__restrict__ F, uint32_t b, uint32_t nb) {
    constexpr int R = 16 * NCT, S = 4 * NCT;
    const int lane = threadIdx.x % 64, g = lane / 16;
    double wa[NCT][S];
    load_rmat<NCT>(W, lane, wa);
    const int64_t ntile = (rows + 15) / 16;
    const int64_t nw = (int64_t)nb * (kBlock / 64);
    int64_t tile = (int64_t)b * (kBlock / 64) + threadIdx.x / 64;
    Run4<float> x[NCT];
    load_rowrun<NCT>(M, tile * 16 + lane % 16, rows, g, x);
    for (; tile < ntile; tile += nw) {
        const int64_t row = tile * 16 + lane % 16;
        Run4<float> xn[NCT];
        load_rowrun<NCT>(M, row + 16 * nw, rows, g, xn);
#pragma unroll
        for (int c = 0; c < NCT; ++c) {
            double4v acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int t = 0; t < S; ++t)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(wa[c][t], x[t / 4][t % 4], acc, 0, 0, 0);
            if (row < rows) store4d(F + row * R + 16 * c + 4 * g, acc);
        }
#pragma unroll
        for (int c = 0; c < NCT; ++c) x[c] = xn[c];
    }
}

template <typename Tout, int NCT>
__global__ __launch_bounds__(kBlock) void k_rowmap_mfma(const float *__restrict__ M, int64_t rows,
                                                        const double *__restrict__ W,
                                                        Tout *__restrict__ F) {
    rowmap_mfma_body<Tout, NCT>(M, rows, W, F, blockIdx.x, gridDim.x);
}

template <typename Tout, int NCT>
__global__ __launch_bounds__(kBlock) void k_rowmap_mfma_group(const RowmapJob *__restrict__ jobs,
                                                              const uint2 *__restrict__ vb) {
    const uint2 v = vb[blockIdx.x];
    const RowmapJob &j = jobs[v.x];
    rowmap_mfma_body<Tout, NCT>(j.M, j.rows, j.W, (Tout *)j.F, v.y, j.nblk);
}

// G[row, s] = -G[row, s] + sum_k F[row, k] H[k, s]  (G holds the MTTKRP on
// entry); partial[block] = sum over the block's rows of <F[row,:], G[row,:]>
// (the entry values).
template <typename T, int NCT>
__global__ __launch_bounds__(kBlock) void k_gd_rows_mfma(float *__restrict__ G,
                                                         const T *__restrict__ F, int64_t rows,
                                                         const double *__restrict__ H,
                                                         double *__restrict__ partial) {
    constexpr int R = 16 * NCT, S = 4 * NCT;
    __shared__ double sh[kBlock];
    const int lane = threadIdx.x % 64, g = lane / 16;
    double wa[NCT][S];
    load_rmat<NCT>(H, lane, wa);
    const int64_t ntile = (rows + 15) / 16;
    const int64_t nw = (int64_t)gridDim.x * (kBlock / 64);
    int64_t tile = (int64_t)blockIdx.x * (kBlock / 64) + threadIdx.x / 64;
    double inner = 0.0;
    Run4<T> f[NCT];
    Run4<float> m[NCT];
    load_rowrun<NCT>(F, tile * 16 + lane % 16, rows, g, f);
    load_rowrun<NCT>((const float *)G, tile * 16 + lane % 16, rows, g, m);
    for (; tile < ntile; tile += nw) {
        const int64_t row = tile * 16 + lane % 16;
        Run4<T> fn[NCT];
        Run4<float> mn[NCT];
        load_rowrun<NCT>(F, row + 16 * nw, rows, g, fn);
        load_rowrun<NCT>((const float *)G, row + 16 * nw, rows, g, mn);
#pragma unroll
        for (int t = 0; t < S; ++t) inner = fma(f[t / 4][t % 4], m[t / 4][t % 4], inner);
#pragma unroll
        for (int c = 0; c < NCT; ++c) {
            double4v acc = {-m[c][0], -m[c][1], -m[c][2], -m[c][3]};
#pragma unroll
            for (int t = 0; t < S; ++t)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(wa[c][t], f[t / 4][t % 4], acc, 0, 0, 0);
            if (row < rows) store4d(G + row * R + 16 * c + 4 * g, acc);
        }
#pragma unroll
        for (int c = 0; c < NCT; ++c) {
            f[c] = fn[c];
            m[c] = mn[c];
        }
    }
    const double tot = block_sum(inner, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// ranks with a matrix-core row kernel; the rows must start 16-byte aligned
// (FP32) or 8-byte aligned (BF16)
bool mfma_rows_ok(int R, const void *a, size_t ea, const void *b, size_t eb) {
    if (!(R == 16 || R == 32 || R == 48 || R == 64)) return false;
    return (uintptr_t)a % (4 * ea) == 0 && (uintptr_t)b % (4 * eb) == 0;
}

unsigned rows_grid_mfma(int64_t rows) {
    const int64_t ntile = (rows + 15) / 16;
    const int64_t want = (ntile + 4 * 4 - 1) / (4 * 4);  // about 4 tiles per wave
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, 2048));
}

template <typename Tout>
void rowmap_mfma(hipStream_t s, const float *M, int64_t rows, int R, const double *W, void *F) {
    const dim3 grid(rows_grid_mfma(rows)), block(kBlock);
    switch (R) {
        case 16: hipLaunchKernelGGL((k_rowmap_mfma<Tout, 1>), grid, block, 0, s, M, rows, W, (Tout *)F); break;
        case 32: hipLaunchKernelGGL((k_rowmap_mfma<Tout, 2>), grid, block, 0, s, M, rows, W, (Tout *)F); break;
        case 48: hipLaunchKernelGGL((k_rowmap_mfma<Tout, 3>), grid, block, 0, s, M, rows, W, (Tout *)F); break;
        default: hipLaunchKernelGGL((k_rowmap_mfma<Tout, 4>), grid, block, 0, s, M, rows, W, (Tout *)F); break;
    }
}

template <typename T>
void gd_rows_mfma(hipStream_t s, float *G, const void *F, int64_t rows, int R, const double *H,
                  double *partial) {
    const dim3 grid(rows_grid_mfma(rows)), block(kBlock);
    const T *Ft = (const T *)F;
    switch (R) {
        case 16: hipLaunchKernelGGL((k_gd_rows_mfma<T, 1>), grid, block, 0, s, G, Ft, rows, H, partial); break;
        case 32: hipLaunchKernelGGL((k_gd_rows_mfma<T, 2>), grid, block, 0, s, G, Ft, rows, H, partial); break;
        case 48: hipLaunchKernelGGL((k_gd_rows_mfma<T, 3>), grid, block, 0, s, G, Ft, rows, H, partial); break;
        default: hipLaunchKernelGGL((k_gd_rows_mfma<T, 4>), grid, block, 0, s, G, Ft, rows, H, partial); break;
    }
}

bool tiled_rows_ok(int R) {  // ranks with a compile-time LDS-tiled row kernel (<= ~51 KB LDS)
    return R == 4 || R == 8 || R == 12 || R == 16 || R == 32 || R == 48;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

int gram_partial_blocks(int64_t rows, int R) {
    const int TS = R <= 16 ? 16 : (R <= 32 ? 32 : 64);
    const int TT = TS / 8;
    const int SL = kBlock / (TT * TT);
    const int64_t want = (rows + (int64_t)SL * 16 - 1) / ((int64_t)SL * 16);
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, 256));
}

GramPlan gram_plan(int64_t rows, int R, const void *F, dfacto_dtype dtype) {
    GramPlan g;
    g.nt = (R + 15) / 16;
    const int bs = g.nt <= 2 ? 1024 : 256;  // 16 waves per block when the registers allow
    // Short factors (batched members): eight 16-row steps per wave, so that a
    // block's fixed costs (combining its waves' sums in LDS, writing its
    // partial R x R block) stay small beside its work.  Longer ones: two, so
    // that a single Gram spreads over enough blocks to fill the device.
    const int64_t per_blk = 16 * (rows < 65536 ? 8 : 2) * (bs / 64);
    const int64_t want = (rows + per_blk - 1) / per_blk;
    g.nblk = (int)std::max<int64_t>(1, std::min<int64_t>(want, 256));
    const size_t es = dtype == DFACTO_F32 ? 4 : 2;
    g.vec = R == 32 && (uintptr_t)F % (2 * es) == 0;
    return g;
}

// the partial-sum buffer of the stream the Gram is launched on
static dfacto_ctx::Slot gram_slot(const dfacto_ctx *ctx) {
    return (ctx->side && ctx->stream == ctx->side) ? dfacto_ctx::kPartialSide
                                                   : dfacto_ctx::kPartial;
}

void launch_gram(dfacto_ctx *ctx, const void *F, dfacto_dtype dtype, int64_t rows, int R,
                 double *G) {
    hipStream_t s = ctx->stream;
    if (R <= 16 * kMfmaMaxTiles) {
        const GramPlan gp = gram_plan(rows, R, F, dtype);
        const int nt = gp.nt, nblk = gp.nblk;
        const bool vec2 = gp.vec;
        double *part = (double *)ws_get(ctx, gram_slot(ctx),
                                        sizeof(double) * 256 * (size_t)R * R);
#define GM(T, NTV, V)                                                                              \
    hipLaunchKernelGGL((k_gram_mfma<T, NTV, (NTV <= 2 ? 1024 : 256), V>), dim3(nblk),              \
                       dim3(NTV <= 2 ? 1024 : 256), 0, s, (const T *)F, rows, R, part)
        if (dtype == DFACTO_F32) {
            if (nt == 1) GM(float, 1, false);
            else if (nt == 2 && vec2) GM(float, 2, true);
            else if (nt == 2) GM(float, 2, false);
            else if (nt == 3) GM(float, 3, false);
            else GM(float, 4, false);
        } else {
            if (nt == 1) GM(uint16_t, 1, false);
            else if (nt == 2 && vec2) GM(uint16_t, 2, true);
            else if (nt == 2) GM(uint16_t, 2, false);
            else if (nt == 3) GM(uint16_t, 3, false);
            else GM(uint16_t, 4, false);
        }
#undef GM
        hipLaunchKernelGGL(k_gram_reduce, dim3((R * R + 15) / 16), dim3(kBlock), 0, s, part, nblk, R,
                           G);
        DF_LAUNCHED();
        return;
    }
    const int TS = R <= 16 ? 16 : (R <= 32 ? 32 : 64);
    const int nt = (R + TS - 1) / TS;
    const int nblk = gram_partial_blocks(rows, R);
    // sized for the largest block count so that the buffer never moves between calls
    double *part = (double *)ws_get(ctx, gram_slot(ctx), sizeof(double) * 256 * (size_t)R * R);
    dim3 grid(nblk, nt * nt);
    const int vec = vec_rows(F, R, dtype == DFACTO_F32 ? 4 : 2);
#define GRAM_LAUNCH(T, TSV)                                                                   \
    hipLaunchKernelGGL((k_gram_partial<T, TSV>), grid, dim3(kBlock), 0, s, (const T *)F, rows, R, \
                       vec, part)
    if (dtype == DFACTO_F32) {
        if (TS == 16) GRAM_LAUNCH(float, 16);
        else if (TS == 32) GRAM_LAUNCH(float, 32);
        else GRAM_LAUNCH(float, 64);
    } else {
        if (TS == 16) GRAM_LAUNCH(uint16_t, 16);
        else if (TS == 32) GRAM_LAUNCH(uint16_t, 32);
        else GRAM_LAUNCH(uint16_t, 64);
    }
#undef GRAM_LAUNCH
    hipLaunchKernelGGL(k_gram_reduce, dim3((R * R + 15) / 16), dim3(kBlock), 0, s, part, nblk, R, G);
    DF_LAUNCHED();
}

void launch_hadamard(dfacto_ctx *ctx, int R, const double *Gp, const double *Gq, double reg,
                     double *H) {
    hipLaunchKernelGGL(k_hadamard, dim3((R * R + kBlock - 1) / kBlock), dim3(kBlock), 0, ctx->stream,
                       R, Gp, Gq, reg, H);
    DF_LAUNCHED();
}

void launch_solve(dfacto_ctx *ctx, int R, const double *Gp, const double *Gq, double reg,
                  double *Hinv, double *scratch, int *flag) {
    if (R <= kSolveSmemMaxR)
        hipLaunchKernelGGL(k_solve<true>, dim3(1), dim3(kBlock), sizeof(double) * 3 * R * R,
                           ctx->stream, R, Gp, Gq, reg, Hinv, scratch, flag);
    else
        hipLaunchKernelGGL(k_solve<false>, dim3(1), dim3(kBlock), 0, ctx->stream, R, Gp, Gq, reg,
                           Hinv, scratch, flag);
    DF_LAUNCHED();
}

void launch_als_lambda(dfacto_ctx *ctx, int R, int mode, const double *Hinv, const double *MtM,
                       double *Gn, double *W, double *lambda_out, const double *GA,
                       const double *GB, double normsq, double *fit_out, double *scratch) {
    if (R <= kLambdaSmemMaxR)
        hipLaunchKernelGGL(k_als_lambda<true>, dim3(1), dim3(kBlock),
                           sizeof(double) * (4 * R * R + R), ctx->stream, R, mode, Hinv, MtM, Gn, W,
                           lambda_out, GA, GB, normsq, fit_out, scratch);
    else
        hipLaunchKernelGGL(k_als_lambda<false>, dim3(1), dim3(kBlock), 0, ctx->stream, R, mode,
                           Hinv, MtM, Gn, W, lambda_out, GA, GB, normsq, fit_out, scratch);
    DF_LAUNCHED();
}

static unsigned rows_grid_generic(int64_t rows, int R, int per_pass_elems) {
    const int rpp = std::max(1, per_pass_elems / R);
    const int64_t npass = (rows + rpp - 1) / rpp;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(npass, 8192));
}

static unsigned rows_grid_tiles(int64_t rows, int R) {
    const int64_t nt = (rows + tile_rows(R) - 1) / tile_rows(R);
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(nt, 2048));
}

template <typename Tout, int RC>
void rowmap_tiled(hipStream_t s, const float *M, int64_t rows, const double *W, void *F) {
    hipLaunchKernelGGL((k_rowmap_t<Tout, RC>), dim3(rows_grid_tiles(rows, RC)), dim3(kBlock),
                       tile_lds_bytes(RC), s, M, rows, W, (Tout *)F);
}

template <typename T, int RC>
void gd_rows_tiled(hipStream_t s, float *G, const void *F, int64_t rows, const double *H,
                   double *partial) {
    hipLaunchKernelGGL((k_gd_rows_t<T, RC>), dim3(rows_grid_tiles(rows, RC)), dim3(kBlock),
                       tile_lds_bytes(RC), s, G, (const T *)F, rows, H, partial);
}

// Dispatch a tiled row kernel on the compile-time rank; false if R has none.
template <template <typename, int> class K, typename T, typename... A>
bool dispatch_tiled(int R, A... args) {
    switch (R) {
        case 4: K<T, 4>::run(args...); return true;
        case 8: K<T, 8>::run(args...); return true;
        case 12: K<T, 12>::run(args...); return true;
        case 16: K<T, 16>::run(args...); return true;
        case 32: K<T, 32>::run(args...); return true;
        case 48: K<T, 48>::run(args...); return true;
        default: return false;
    }
}
template <typename T, int RC>
struct RowmapK {
    static void run(hipStream_t s, const float *M, int64_t rows, const double *W, void *F) {
        rowmap_tiled<T, RC>(s, M, rows, W, F);
    }
};
template <typename T, int RC>
struct GdRowsK {
    static void run(hipStream_t s, float *G, const void *F, int64_t rows, const double *H,
                    double *partial) {
        gd_rows_tiled<T, RC>(s, G, F, rows, H, partial);
    }
};

void launch_rowmap(dfacto_ctx *ctx, const float *M, int64_t rows, int R, const double *W, void *F,
                   dfacto_dtype dtype) {
    if (rows <= 0) return;
    hipStream_t s = ctx->stream;
    const size_t ef = dtype == DFACTO_F32 ? 4 : 2;
    if (mfma_rows_ok(R, M, 4, F, ef)) {
        if (dtype == DFACTO_F32) rowmap_mfma<float>(s, M, rows, R, W, F);
        else rowmap_mfma<uint16_t>(s, M, rows, R, W, F);
        DF_LAUNCHED();
        return;
    }
    const bool done = dtype == DFACTO_F32
                          ? dispatch_tiled<RowmapK, float>(R, s, M, rows, W, F)
                          : dispatch_tiled<RowmapK, uint16_t>(R, s, M, rows, W, F);
    if (!done) {
        const unsigned g = rows_grid_generic(rows, R, kBlock * 4);
        if (dtype == DFACTO_F32)
            hipLaunchKernelGGL(k_rowmap_g<float>, dim3(g), dim3(kBlock), 0, s, M, rows, R, W,
                               (float *)F);
        else
            hipLaunchKernelGGL(k_rowmap_g<uint16_t>, dim3(g), dim3(kBlock), 0, s, M, rows, R, W,
                               (uint16_t *)F);
    }
    DF_LAUNCHED();
}

int gd_rows_partials(int64_t rows, int R, const float *G, const void *F, dfacto_dtype dtype) {
    if (mfma_rows_ok(R, G, 4, F, dtype == DFACTO_F32 ? 4 : 2)) return (int)rows_grid_mfma(rows);
    return (int)(tiled_rows_ok(R) ? rows_grid_tiles(rows, R)
                                  : rows_grid_generic(rows, R, kBlock * 2));
}

void launch_gd_rows(dfacto_ctx *ctx, float *G, const void *F, dfacto_dtype dtype, int64_t rows,
                    int R, const double *H, double *inner_partial) {
    if (rows <= 0) return;
    hipStream_t s = ctx->stream;
    if (mfma_rows_ok(R, G, 4, F, dtype == DFACTO_F32 ? 4 : 2)) {
        if (dtype == DFACTO_F32) gd_rows_mfma<float>(s, G, F, rows, R, H, inner_partial);
        else gd_rows_mfma<uint16_t>(s, G, F, rows, R, H, inner_partial);
        DF_LAUNCHED();
        return;
    }
    const bool done = dtype == DFACTO_F32
                          ? dispatch_tiled<GdRowsK, float>(R, s, G, F, rows, H, inner_partial)
                          : dispatch_tiled<GdRowsK, uint16_t>(R, s, G, F, rows, H, inner_partial);
    if (!done) {
        const unsigned g = (unsigned)gd_rows_partials(rows, R, G, F, dtype);
        if (dtype == DFACTO_F32)
            hipLaunchKernelGGL(k_gd_rows_g<float>, dim3(g), dim3(kBlock), 0, s, G,
                               (const float *)F, rows, R, H, inner_partial);
        else
            hipLaunchKernelGGL(k_gd_rows_g<uint16_t>, dim3(g), dim3(kBlock), 0, s, G,
                               (const uint16_t *)F, rows, R, H, inner_partial);
    }
    DF_LAUNCHED();
}

void launch_gd_f(dfacto_ctx *ctx, int R, const double *GA, const double *GB, const double *GC,
                 const double *inner_partial, int npartial, double normsq, double reg,
                 double *f_out) {
    hipLaunchKernelGGL(k_gd_f, dim3(1), dim3(kBlock), 0, ctx->stream, R, GA, GB, GC, inner_partial,
                       npartial, normsq, reg, f_out);
    DF_LAUNCHED();
}

unsigned stream_grid(int64_t n) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, 4096));
}

void launch_trial_factor(dfacto_ctx *ctx, const void *F, const float *G, double alpha, void *out,
                         dfacto_dtype dtype, int64_t n) {
    if (n <= 0) return;
    if (dtype == DFACTO_F32)
        hipLaunchKernelGGL(k_trial_factor<float>, dim3(stream_grid(n)), dim3(kBlock), 0,
                           ctx->stream, (const float *)F, G, alpha, (float *)out, n);
    else
        hipLaunchKernelGGL(k_trial_factor<uint16_t>, dim3(stream_grid(n)), dim3(kBlock), 0,
                           ctx->stream, (const uint16_t *)F, G, alpha, (uint16_t *)out, n);
    DF_LAUNCHED();
}

void launch_sumsq3(dfacto_ctx *ctx, const float *const x[3], const int64_t n[3], double *part,
                   double *out) {
    for (int m = 0; m < 3; ++m)
        hipLaunchKernelGGL(k_sumsq_f32, dim3(kSumsqBlocks), dim3(kBlock), 0, ctx->stream, x[m],
                           n[m], part + m * kSumsqBlocks);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kBlock), 0, ctx->stream, part,
                       3 * kSumsqBlocks, out);
    DF_LAUNCHED();
}

// workgroups of `block` threads of `kernel` that one CU holds at once (>= 1)
template <typename K>
int resident_blocks(K kernel, int block) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, block, 0) != hipSuccess || n < 1)
        n = 1;
    return n;
}

void launch_joint_rows(dfacto_ctx *ctx, const dfacto_tensor *Y, int m, int64_t nrows,
                       const void *Fmid, const void *Fleaf, int R, const float *M,
                       const double *H, double mu, double lam, const double *Pinv, double ws,
                       const int *pflag, void *out, dfacto_dtype dtype, int *flag, double *part) {
    if (nrows <= 0) return;
    hipStream_t s = ctx->stream;
    const uint2 *st = Y->mode[m].stream;
    // persistent: the grid is what the device holds at once, so no
    // workgroup waits for a second round
    static const int occ_f32 = resident_blocks(k_joint_rows<float>, 64);
    static const int occ_bf16 = resident_blocks(k_joint_rows<uint16_t>, 64);
    const int occ = dtype == DFACTO_F32 ? occ_f32 : occ_bf16;
    const unsigned grid =
        (unsigned)std::min<int64_t>(nrows, (int64_t)std::max(1, ctx->num_cu) * occ);
    const int64_t nseg = Y->nseg[m], nheavy = Y->nheavy[m];
    const unsigned gseg = (unsigned)std::max<int64_t>(1, std::min<int64_t>(nseg, 1 << 20));
    const unsigned ghv = (unsigned)std::max<int64_t>(1, std::min<int64_t>(nheavy, 1 << 20));
#define DF_JOINT(T)                                                                            \
    hipLaunchKernelGGL(k_joint_rows<T>, dim3(grid), dim3(64), 0, s, st, Y->row_range[m], nrows, \
                       (const T *)Fmid, (const T *)Fleaf, R, M, H, mu, lam, Pinv, ws, pflag,   \
                       (T *)out, flag);                                                        \
    if (nseg > 0) {                                                                            \
        hipLaunchKernelGGL(k_joint_segments<T>, dim3(gseg), dim3(64), 0, s, st,               \
                           Y->seg_range[m], nseg, (const T *)Fmid, (const T *)Fleaf, R, part); \
        hipLaunchKernelGGL(k_joint_heavy<T>, dim3(ghv), dim3(64), 0, s, Y->heavy[m], nheavy,  \
                           R, part, M, H, mu, lam, (T *)out, flag);                            \
    }
    if (dtype == DFACTO_F32) {
        DF_JOINT(float)
    } else {
        DF_JOINT(uint16_t)
    }
#undef DF_JOINT
    DF_LAUNCHED();
}

void launch_joint_combine(dfacto_ctx *ctx, float *G, const void *F, const float *RY, double mu,
                          double lam, int64_t n, dfacto_dtype dtype) {
    if (n <= 0) return;
    if (dtype == DFACTO_F32)
        hipLaunchKernelGGL(k_joint_combine<float>, dim3(stream_grid(n)), dim3(kBlock), 0,
                           ctx->stream, G, (const float *)F, RY, mu, lam, n);
    else
        hipLaunchKernelGGL(k_joint_combine<uint16_t>, dim3(stream_grid(n)), dim3(kBlock), 0,
                           ctx->stream, G, (const uint16_t *)F, RY, mu, lam, n);
    DF_LAUNCHED();
}

uint32_t fit_blocks(int64_t rows, int R) {
    const int64_t n = rows * (int64_t)R;
    return (uint32_t)std::min<int64_t>(64, std::max<int64_t>(1, (n + 16383) / 16384));
}

void launch_fit_stored(dfacto_ctx *ctx, const void *F, dfacto_dtype dtype, const float *M,
                       int64_t rows, int R, const double *lambda, const double *GA,
                       const double *GB, const double *GC, double normsq, double *part,
                       double *fit) {
    const uint32_t nb = fit_blocks(rows, R);
    if (dtype == DFACTO_F32)
        hipLaunchKernelGGL(k_wdot<float>, dim3(nb), dim3(kBlock), 0, ctx->stream,
                           (const float *)F, M, rows, R, lambda, part);
    else
        hipLaunchKernelGGL(k_wdot<uint16_t>, dim3(nb), dim3(kBlock), 0, ctx->stream,
                           (const uint16_t *)F, M, rows, R, lambda, part);
    hipLaunchKernelGGL(k_fit_finish, dim3(1), dim3(kBlock), 0, ctx->stream, R, lambda, GA, GB, GC,
                       part, nb, normsq, fit);
    DF_LAUNCHED();
}

void launch_fit_group(dfacto_ctx *ctx, dfacto_dtype dtype, const FitJob *d_jobs, uint32_t n,
                      const uint2 *d_items, uint32_t nitems) {
    if (nitems > 0) {
        if (dtype == DFACTO_F32)
            hipLaunchKernelGGL(k_wdot_group<float>, dim3(nitems), dim3(kBlock), 0, ctx->stream,
                               d_jobs, d_items);
        else
            hipLaunchKernelGGL(k_wdot_group<uint16_t>, dim3(nitems), dim3(kBlock), 0,
                               ctx->stream, d_jobs, d_items);
    }
    hipLaunchKernelGGL(k_fit_finish_group, dim3(n), dim3(kBlock), 0, ctx->stream, d_jobs);
    DF_LAUNCHED();
}

void launch_dot_parts(dfacto_ctx *ctx, const void *F, const float *X, int64_t n, double *part,
                      dfacto_dtype dtype) {
    if (dtype == DFACTO_F32)
        hipLaunchKernelGGL(k_dot_parts<float>, dim3(kSumsqBlocks), dim3(kBlock), 0, ctx->stream,
                           (const float *)F, X, n, part);
    else
        hipLaunchKernelGGL(k_dot_parts<uint16_t>, dim3(kSumsqBlocks), dim3(kBlock), 0,
                           ctx->stream, (const uint16_t *)F, X, n, part);
    DF_LAUNCHED();
}

void launch_joint_f(dfacto_ctx *ctx, const double *ft, const double *GA, const double *GB,
                    const double *GC, int R, const double *part, int npart, double normsq_y,
                    double mu, double lam, double *f) {
    hipLaunchKernelGGL(k_joint_f, dim3(1), dim3(kBlock), 0, ctx->stream, ft, GA, GB, GC, R, part,
                       npart, normsq_y, mu, lam, f);
    DF_LAUNCHED();
}

// ---- grouped launches (many tensors, one launch per kernel class) ---------
void launch_gram_group(dfacto_ctx *ctx, dfacto_dtype dtype, int nt, bool vec,
                       const GramJob *d_jobs, const uint2 *d_vb, uint32_t nvb) {
    if (nvb == 0) return;
    hipStream_t s = ctx->stream;
#define GMG(T, NTV, V)                                                                         \
    hipLaunchKernelGGL((k_gram_mfma_group<T, NTV, (NTV <= 2 ? 1024 : 256), V>), dim3(nvb),     \
                       dim3(NTV <= 2 ? 1024 : 256), 0, s, d_jobs, d_vb)
    if (dtype == DFACTO_F32) {
        if (nt == 1) GMG(float, 1, false);
        else if (nt == 2 && vec) GMG(float, 2, true);
        else if (nt == 2) GMG(float, 2, false);
        else if (nt == 3) GMG(float, 3, false);
        else GMG(float, 4, false);
    } else {
        if (nt == 1) GMG(uint16_t, 1, false);
        else if (nt == 2 && vec) GMG(uint16_t, 2, true);
        else if (nt == 2) GMG(uint16_t, 2, false);
        else if (nt == 3) GMG(uint16_t, 3, false);
        else GMG(uint16_t, 4, false);
    }
#undef GMG
    DF_LAUNCHED();
}

uint32_t gram_reduce_blocks(int R) { return (uint32_t)((R * R + 15) / 16); }

void launch_gram_reduce_group(dfacto_ctx *ctx, const GramJob *d_jobs, const uint2 *d_vb,
                              uint32_t nvb) {
    if (nvb == 0) return;
    hipLaunchKernelGGL(k_gram_reduce_group, dim3(nvb), dim3(kBlock), 0, ctx->stream, d_jobs, d_vb);
    DF_LAUNCHED();
}

void launch_solve_group(dfacto_ctx *ctx, int maxR, const SolveJob *d_jobs, uint32_t n) {
    if (n == 0) return;
    if (maxR <= kSolveSmemMaxR)
        hipLaunchKernelGGL(k_solve_group<true>, dim3(n), dim3(kBlock),
                           sizeof(double) * 3 * maxR * maxR, ctx->stream, d_jobs);
    else
        hipLaunchKernelGGL(k_solve_group<false>, dim3(n), dim3(kBlock), 0, ctx->stream, d_jobs);
    DF_LAUNCHED();
}

void launch_lambda_group(dfacto_ctx *ctx, int maxR, const LambdaJob *d_jobs, uint32_t n) {
    if (n == 0) return;
    if (maxR <= kLambdaSmemMaxR)
        hipLaunchKernelGGL(k_als_lambda_group<true>, dim3(n), dim3(kBlock),
                           sizeof(double) * (4 * maxR * maxR + maxR), ctx->stream, d_jobs);
    else
        hipLaunchKernelGGL(k_als_lambda_group<false>, dim3(n), dim3(kBlock), 0, ctx->stream,
                           d_jobs);
    DF_LAUNCHED();
}

RowmapPlan rowmap_plan(int R, const float *M, const void *F, dfacto_dtype dtype, int64_t rows) {
    RowmapPlan p;
    if (mfma_rows_ok(R, M, 4, F, dtype == DFACTO_F32 ? 4 : 2)) {
        p.kind = RowmapPlan::kMfma;
        p.nblk = rows_grid_mfma(rows);
    } else if (tiled_rows_ok(R)) {
        p.kind = RowmapPlan::kTiled;
        p.nblk = rows_grid_tiles(rows, R);
    } else {
        p.kind = RowmapPlan::kGeneric;
        p.nblk = 0;
    }
    return p;
}

void launch_rowmap_group(dfacto_ctx *ctx, dfacto_dtype dtype, int kind, int R,
                         const RowmapJob *d_jobs, const uint2 *d_vb, uint32_t nvb) {
    if (nvb == 0) return;
    hipStream_t s = ctx->stream;
    const dim3 grid(nvb), block(kBlock);
    auto mfma = [&](auto tag) {
        using Tout = decltype(tag);
        switch (R) {
            case 16: hipLaunchKernelGGL((k_rowmap_mfma_group<Tout, 1>), grid, block, 0, s, d_jobs, d_vb); break;
            case 32: hipLaunchKernelGGL((k_rowmap_mfma_group<Tout, 2>), grid, block, 0, s, d_jobs, d_vb); break;
            case 48: hipLaunchKernelGGL((k_rowmap_mfma_group<Tout, 3>), grid, block, 0, s, d_jobs, d_vb); break;
            case 64: hipLaunchKernelGGL((k_rowmap_mfma_group<Tout, 4>), grid, block, 0, s, d_jobs, d_vb); break;
            default: throw Error{DFACTO_E_UNSUPPORTED, "no grouped row map for this rank"};
        }
    };
    auto tiled = [&](auto tag) {
        using Tout = decltype(tag);
        const size_t lds = tile_lds_bytes(R);
        switch (R) {
            case 4: hipLaunchKernelGGL((k_rowmap_t_group<Tout, 4>), grid, block, lds, s, d_jobs, d_vb); break;
            case 8: hipLaunchKernelGGL((k_rowmap_t_group<Tout, 8>), grid, block, lds, s, d_jobs, d_vb); break;
            case 12: hipLaunchKernelGGL((k_rowmap_t_group<Tout, 12>), grid, block, lds, s, d_jobs, d_vb); break;
            case 16: hipLaunchKernelGGL((k_rowmap_t_group<Tout, 16>), grid, block, lds, s, d_jobs, d_vb); break;
            case 32: hipLaunchKernelGGL((k_rowmap_t_group<Tout, 32>), grid, block, lds, s, d_jobs, d_vb); break;
            case 48: hipLaunchKernelGGL((k_rowmap_t_group<Tout, 48>), grid, block, lds, s, d_jobs, d_vb); break;
            default: throw Error{DFACTO_E_UNSUPPORTED, "no grouped row map for this rank"};
        }
    };
    if (kind == RowmapPlan::kMfma) {
        if (dtype == DFACTO_F32) mfma(float{});
        else mfma(uint16_t{});
    } else if (kind == RowmapPlan::kTiled) {
        if (dtype == DFACTO_F32) tiled(float{});
        else tiled(uint16_t{});
    } else {
        throw Error{DFACTO_E_UNSUPPORTED, "no grouped row map for this rank"};
    }
    DF_LAUNCHED();
}

}  // namespace dfacto
