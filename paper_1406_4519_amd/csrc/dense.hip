// dense.hip -- the small dense FP64 parts of CP-ALS and GD (Appendix B and C)
//
//  * Gram F^T F of a factor or of an MTTKRP result, FP64 accumulation
//    (tiled, fixed-order two-pass reduction).
//  * H = G_p * G_q + reg I (Appendix A: (A kr B)^T (A kr B) = A^T A * B^T B,
//    ridge term of the regularized update).
//  * One-workgroup FP64 solve: Cholesky inverse of H, or the Moore-Penrose
//    pseudo-inverse from a parallel cyclic Jacobi eigen-decomposition when a
//    pivot shows H is numerically singular.
//  * Column norms, the new Gram and the fit from R x R algebra: with
//    Fhat = M H^-1,  Fhat^T Fhat = H^-1 (M^T M) H^-1, so
//    lambda_r^2 = [H^-1 M^T M H^-1]_rr and  <X, Xhat> = <Fhat, M> =
//    trace(H^-1 M^T M) for the last mode; ||Xhat||^2 = lambda^T (G_A * G_B *
//    G_C) lambda.
//  * Row maps F = M W (W = H^-1 diag(1/lambda)) and the GD gradient
//    -M + F H.
#include <hip/hip_runtime.h>

#include <cfloat>

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

// ---------------------------------------------------------------------------
// Gram: partial[b][r][s] = sum over the rows of block b of F[row][r] F[row][s]
// grid.x: row blocks (grid-stride over row tiles), grid.y: TSxTS tiles.
// 256 threads as 16 x 16, each an MT x MT micro-tile (TS = 16 MT).
// ---------------------------------------------------------------------------
template <typename T, int TS>
__global__ __launch_bounds__(kBlock) void k_gram_partial(const T *__restrict__ F, int64_t rows,
                                                         int R, double *__restrict__ part) {
    constexpr int MT = TS / 16;
    constexpr int kGramRows = 2048 / TS;  // rows staged per tile
    __shared__ double sa[kGramRows][TS + 1];
    __shared__ double sb[kGramRows][TS + 1];
    const int nt = (R + TS - 1) / TS;
    const int rt = blockIdx.y / nt, ct = blockIdx.y % nt;
    const int r0 = rt * TS, c0 = ct * TS;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    double acc[MT][MT];
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int b = 0; b < MT; ++b) acc[a][b] = 0.0;
    const int64_t ntile = (rows + kGramRows - 1) / kGramRows;
    for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        const int64_t base = tile * kGramRows;
        __syncthreads();
        for (int e = threadIdx.x; e < kGramRows * TS; e += kBlock) {
            const int rr = e / TS, cc = e % TS;
            const int64_t row = base + rr;
            const bool okr = row < rows;
            sa[rr][cc] = (okr && r0 + cc < R) ? ld<T>(F, row * R + r0 + cc) : 0.0;
            sb[rr][cc] = (okr && c0 + cc < R) ? ld<T>(F, row * R + c0 + cc) : 0.0;
        }
        __syncthreads();
        for (int rr = 0; rr < kGramRows; ++rr) {
            double x[MT], y[MT];
#pragma unroll
            for (int a = 0; a < MT; ++a) x[a] = sa[rr][ty * MT + a];
#pragma unroll
            for (int b = 0; b < MT; ++b) y[b] = sb[rr][tx * MT + b];
#pragma unroll
            for (int a = 0; a < MT; ++a)
#pragma unroll
                for (int b = 0; b < MT; ++b) acc[a][b] = fma(x[a], y[b], acc[a][b]);
        }
    }
    double *pb = part + (size_t)blockIdx.x * R * R;
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int b = 0; b < MT; ++b) {
            const int r = r0 + ty * MT + a, c = c0 + tx * MT + b;
            if (r < R && c < R) pb[r * R + c] = acc[a][b];
        }
}

__global__ void k_gram_reduce(const double *__restrict__ part, int nblk, int R,
                              double *__restrict__ G) {
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= R * R) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * R * R + e];
    G[e] = s;
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

// ---------------------------------------------------------------------------
// one-workgroup solve.  scratch: 4 R^2 doubles (H, L / A, Linv / V, spare).
// flag[0] = 1 when the pseudo-inverse path was taken.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_solve(int R, const double *__restrict__ Gp,
                                                  const double *__restrict__ Gq, double reg,
                                                  double *__restrict__ Hinv,
                                                  double *__restrict__ scratch, int *flag) {
    __shared__ double sh[kBlock];
    __shared__ int s_fail;
    __shared__ double s_c[kBlock], s_s[kBlock];
    __shared__ int s_p[kBlock], s_q[kBlock];
    const int tid = threadIdx.x;
    const int RR = R * R;
    double *H = scratch, *L = scratch + RR, *Li = scratch + 2 * RR;
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
    // Cholesky H = L L^T, column by column
    for (int j = 0; j < R && !s_fail; ++j) {
        if (tid == 0) {
            double d = H[j * R + j];
            for (int k = 0; k < j; ++k) d -= L[j * R + k] * L[j * R + k];
            if (!(d > tol)) s_fail = 1;
            else L[j * R + j] = sqrt(d);
        }
        __syncthreads();
        if (s_fail) break;
        const double ljj = L[j * R + j];
        for (int i = j + 1 + tid; i < R; i += kBlock) {
            double s = H[i * R + j];
            for (int k = 0; k < j; ++k) s -= L[i * R + k] * L[j * R + k];
            L[i * R + j] = s / ljj;
        }
        __syncthreads();
    }
    if (!s_fail) {
        // Linv = L^{-1} (lower triangular), one column per thread
        for (int c = tid; c < R; c += kBlock) {
            for (int i = c; i < R; ++i) {
                double s = (i == c) ? 1.0 : 0.0;
                for (int k = c; k < i; ++k) s -= L[i * R + k] * Li[k * R + c];
                Li[i * R + c] = s / L[i * R + i];
            }
        }
        __syncthreads();
        // H^{-1} = Linv^T Linv
        for (int e = tid; e < RR; e += kBlock) {
            const int r = e / R, s = e % R;
            const int k0 = r > s ? r : s;
            double acc = 0.0;
            for (int k = k0; k < R; ++k) acc += Li[k * R + r] * Li[k * R + s];
            Hinv[e] = acc;
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

// ---------------------------------------------------------------------------
// lambda, new Gram, W and (last mode) fit -- one workgroup.
// scratch T1 = MtM H^-1 (R^2), S = H^-1 T1 (R^2).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_als_lambda(
    int R, int mode, const double *__restrict__ Hinv, const double *__restrict__ MtM,
    double *__restrict__ Gn, double *__restrict__ W, double *__restrict__ lambda_out,
    const double *__restrict__ GA, const double *__restrict__ GB, double normsq,
    double *__restrict__ fit_out, double *__restrict__ scratch) {
    __shared__ double sh[kBlock];
    const int tid = threadIdx.x;
    const int RR = R * R;
    double *T1 = scratch, *S = scratch + RR, *lam = scratch + 2 * RR;
    for (int e = tid; e < RR; e += kBlock) {
        const int r = e / R, s = e % R;
        double acc = 0.0;
        for (int k = 0; k < R; ++k) acc += MtM[r * R + k] * Hinv[k * R + s];
        T1[e] = acc;
    }
    __syncthreads();
    for (int e = tid; e < RR; e += kBlock) {
        const int r = e / R, s = e % R;
        double acc = 0.0;
        for (int k = 0; k < R; ++k) acc += Hinv[r * R + k] * T1[k * R + s];
        S[e] = acc;
    }
    __syncthreads();
    for (int r = tid; r < R; r += kBlock) {
        const double d = S[r * R + r];
        lam[r] = d > 0.0 ? sqrt(d) : 0.0;
        lambda_out[r] = lam[r];
    }
    __syncthreads();
    for (int e = tid; e < RR; e += kBlock) {
        const int r = e / R, s = e % R;
        const double lr = lam[r], ls = lam[s];
        Gn[e] = (lr > 0.0 && ls > 0.0) ? S[e] / (lr * ls) : 0.0;
        W[e] = ls > 0.0 ? Hinv[e] / ls : 0.0;
    }
    if (mode != 2) return;
    __syncthreads();
    double in = 0.0, xh = 0.0;
    for (int e = tid; e < RR; e += kBlock) {
        const int r = e / R, s = e % R;
        in += Hinv[e] * MtM[e];
        xh += lam[r] * lam[s] * GA[e] * GB[e] * Gn[e];
    }
    in = block_sum(in, sh);
    xh = block_sum(xh, sh);
    if (tid == 0) {
        double res2 = normsq + xh - 2.0 * in;
        if (res2 < 0.0) res2 = 0.0;
        *fit_out = normsq > 0.0 ? 1.0 - sqrt(res2) / sqrt(normsq) : 0.0;
    }
}

// ---------------------------------------------------------------------------
// row maps.  A block handles kRowsPerPass rows per pass; the rows of the
// input and the R x R matrix are staged in LDS (W only when R <= 64).
// ---------------------------------------------------------------------------
constexpr int kLdsMatMaxR = 64;

// F[row, s] = sum_r M[row, r] W[r, s]
template <typename Tout>
__global__ __launch_bounds__(kBlock) void k_rowmap(const float *__restrict__ M, int64_t rows,
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

// G[row, s] = -G[row, s] + sum_r F[row, r] H[r, s]   (G holds the MTTKRP);
// partial[block] = sum over the block's rows of <F[row,:], M[row,:]>.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gd_rows(float *__restrict__ G, const T *__restrict__ F,
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

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

void launch_gram(dfacto_ctx *ctx, const void *F, dfacto_dtype dtype, int64_t rows, int R,
                 double *G) {
    hipStream_t s = ctx->stream;
    const int TS = R <= 16 ? 16 : (R <= 32 ? 32 : 64);
    const int nt = (R + TS - 1) / TS;
    const int64_t ntile = (rows + (2048 / TS) - 1) / (2048 / TS);
    int64_t cap = (int64_t)(4 << 20) / ((int64_t)R * R);
    cap = std::max<int64_t>(1, std::min<int64_t>(cap, 1024));
    const int nblk = (int)std::max<int64_t>(1, std::min<int64_t>(ntile, cap));
    // sized for the largest row count so that the buffer never moves between calls
    double *part = (double *)ws_get(ctx, dfacto_ctx::kPartial, sizeof(double) * (size_t)cap * R * R);
    dim3 grid(nblk, nt * nt);
#define GRAM_LAUNCH(T, TSV)                                                                   \
    hipLaunchKernelGGL((k_gram_partial<T, TSV>), grid, dim3(kBlock), 0, s, (const T *)F, rows, R, \
                       part)
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
    hipLaunchKernelGGL(k_gram_reduce, dim3((R * R + kBlock - 1) / kBlock), dim3(kBlock), 0, s, part,
                       nblk, R, G);
    DF_HIP(hipGetLastError());
}

void launch_hadamard(dfacto_ctx *ctx, int R, const double *Gp, const double *Gq, double reg,
                     double *H) {
    hipLaunchKernelGGL(k_hadamard, dim3((R * R + kBlock - 1) / kBlock), dim3(kBlock), 0, ctx->stream,
                       R, Gp, Gq, reg, H);
    DF_HIP(hipGetLastError());
}

void launch_solve(dfacto_ctx *ctx, int R, const double *Gp, const double *Gq, double reg,
                  double *Hinv, double *scratch, int *flag) {
    hipLaunchKernelGGL(k_solve, dim3(1), dim3(kBlock), 0, ctx->stream, R, Gp, Gq, reg, Hinv,
                       scratch, flag);
    DF_HIP(hipGetLastError());
}

void launch_als_lambda(dfacto_ctx *ctx, int R, int mode, const double *Hinv, const double *MtM,
                       double *Gn, double *W, double *lambda_out, const double *GA,
                       const double *GB, double normsq, double *fit_out, double *scratch) {
    hipLaunchKernelGGL(k_als_lambda, dim3(1), dim3(kBlock), 0, ctx->stream, R, mode, Hinv, MtM, Gn,
                       W, lambda_out, GA, GB, normsq, fit_out, scratch);
    DF_HIP(hipGetLastError());
}

static unsigned rows_grid(int64_t rows, int R, int per_pass_elems) {
    const int rpp = std::max(1, per_pass_elems / R);
    const int64_t npass = (rows + rpp - 1) / rpp;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(npass, 8192));
}

void launch_rowmap(dfacto_ctx *ctx, const float *M, int64_t rows, int R, const double *W, void *F,
                   dfacto_dtype dtype) {
    if (rows <= 0) return;
    const unsigned g = rows_grid(rows, R, kBlock * 4);
    if (dtype == DFACTO_F32)
        hipLaunchKernelGGL(k_rowmap<float>, dim3(g), dim3(kBlock), 0, ctx->stream, M, rows, R, W,
                           (float *)F);
    else
        hipLaunchKernelGGL(k_rowmap<uint16_t>, dim3(g), dim3(kBlock), 0, ctx->stream, M, rows, R, W,
                           (uint16_t *)F);
    DF_HIP(hipGetLastError());
}

int gd_rows_partials(int64_t rows, int R) { return (int)rows_grid(rows, R, kBlock * 2); }

void launch_gd_rows(dfacto_ctx *ctx, float *G, const void *F, dfacto_dtype dtype, int64_t rows,
                    int R, const double *H, double *inner_partial) {
    if (rows <= 0) return;
    const unsigned g = rows_grid(rows, R, kBlock * 2);
    if (dtype == DFACTO_F32)
        hipLaunchKernelGGL(k_gd_rows<float>, dim3(g), dim3(kBlock), 0, ctx->stream, G,
                           (const float *)F, rows, R, H, inner_partial);
    else
        hipLaunchKernelGGL(k_gd_rows<uint16_t>, dim3(g), dim3(kBlock), 0, ctx->stream, G,
                           (const uint16_t *)F, rows, R, H, inner_partial);
    DF_HIP(hipGetLastError());
}

void launch_gd_f(dfacto_ctx *ctx, int R, const double *GA, const double *GB, const double *GC,
                 const double *inner_partial, int npartial, double normsq, double reg,
                 double *f_out) {
    hipLaunchKernelGGL(k_gd_f, dim3(1), dim3(kBlock), 0, ctx->stream, R, GA, GB, GC, inner_partial,
                       npartial, normsq, reg, f_out);
    DF_HIP(hipGetLastError());
}

}  // namespace dfacto
