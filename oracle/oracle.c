/*
 * oracle.c -- plain FP64 CPU reference for the DFacTo hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can compare the HIP library against an
 * independent, obviously correct computation.  It shares no code, header,
 * table or helper with the GPU path.
 *
 * Everything here is a slow loop over coordinate-format (COO) nonzeros in
 * double precision, written from the definitions in
 *   Choi & Vishwanathan, "DFacTo: Distributed Factorization of Tensors"
 *   (NIPS 2014):
 *   - Section 2.1, eq. (1): the three cyclic flattenings
 *       x_{ijk} = X1[i, j + k*J] = X2[j, k + i*K] = X3[k, i + j*I]   (0-based)
 *   - Appendix A: Khatri-Rao product, Hadamard product, and the identity
 *       (A kr B)^T (A kr B) = A^T A * B^T B
 *   - Lemma 2 (Section 3): column r of X1 (C kr B) equals
 *       [unvec_(K,I)((X2)^T b_r)]^T c_r ,
 *     whose entry i is sum_{j,k} x_{ijk} b_{jr} c_{kr}.  The oracle uses that
 *     element form directly (per nonzero), not the two sparse products.
 *   - Appendix B: CP model with unit-norm columns and weights lambda,
 *     Algorithm 2 (CP-ALS, Gauss-Seidel order A, B, C), the least-squares
 *     update  A <- X1 (C kr B) (C^T C * B^T B + reg I)^{-1}  (ridge form).
 *   - Appendix C: GD objective f = 1/2 ||X - [[A,B,C]]||^2 (+ ridge), and
 *       dF/dA = -X1 (C kr B) + A (C^T C * B^T B + reg I).
 *   - Algorithm 5 (Appendix E, DFacTo with GD): the three gradients at one
 *     point, a backtracking line search, the simultaneous update.
 *   - The joint matrix completion and tensor factorization model (its
 *     objective, per-row gradient and per-row ALS closed form).
 *
 * Mode numbering is 0-based: mode 0 is the paper's mode 1 (output rows i),
 * mode 1 is the paper's mode 2 (rows j), mode 2 the paper's mode 3 (rows k).
 *
 * Duplicate coordinates are summed (the paper does not say; linear algebra
 * on a sparse tensor with repeated coordinates sums them).
 *
 * Threads (oracle_config): the same loops can be spread over host threads
 * for full-size checks and the all-cores CPU baseline.  Only independent
 * work is split -- disjoint output rows of an MTTKRP (each row still adds
 * its nonzeros in input order), disjoint Gram entries, rows of a solve,
 * columns of a norm -- and every sum keeps its serial order, so results are
 * bitwise the same for any thread count.
 */
#define _POSIX_C_SOURCE 200809L
#include <float.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* optional threads                                                    */
/* ------------------------------------------------------------------ */

#define MAX_THREADS 256
static int g_threads = 1;  /* worker threads of the loops below */
static int g_distinct = 0; /* caller guarantees distinct coordinates */

/* threads: worker threads (1 = serial).  assume_distinct != 0: the caller
 * guarantees that no coordinate repeats, so merging duplicates is the
 * identity and ||X||^2 is the sum of squared values in input order (no
 * sort of the nonzeros). */
void oracle_config(int threads, int assume_distinct)
{
    g_threads = threads < 1 ? 1 : (threads > MAX_THREADS ? MAX_THREADS : threads);
    g_distinct = assume_distinct != 0;
}

typedef void (*range_fn)(void *arg, int64_t lo, int64_t hi);
typedef struct {
    range_fn fn;
    void *arg;
    int64_t lo, hi;
} par_job;

static void *par_run(void *p)
{
    par_job *j = (par_job *)p;
    j->fn(j->arg, j->lo, j->hi);
    return NULL;
}

/* fn over [0, n) in g_threads contiguous ranges, one thread each. */
static void par_for(int64_t n, range_fn fn, void *arg)
{
    int T = g_threads;
    if ((int64_t)T > n) T = n > 1 ? (int)n : 1;
    if (T <= 1) {
        fn(arg, 0, n);
        return;
    }
    pthread_t th[MAX_THREADS];
    par_job jb[MAX_THREADS];
    for (int t = 0; t < T; ++t) {
        jb[t].fn = fn;
        jb[t].arg = arg;
        jb[t].lo = n * t / T;
        jb[t].hi = n * (t + 1) / T;
        if (pthread_create(&th[t], NULL, par_run, &jb[t]) != 0) {
            par_run(&jb[t]); /* no thread: run it here */
            th[t] = pthread_self();
        }
    }
    for (int t = 0; t < T; ++t)
        if (!pthread_equal(th[t], pthread_self())) pthread_join(th[t], NULL);
}

/* ------------------------------------------------------------------ */
/* small dense helpers (row-major)                                     */
/* ------------------------------------------------------------------ */

/* G = F^T F for F (rows x R): G[r][s] = sum over n (in order) of
 * F[n][r] F[n][s].  Threads take disjoint rows r of G. */
typedef struct {
    int64_t rows;
    int R;
    const double *F;
    double *G;
} gram_arg;

static void gram_part(void *p, int64_t r0, int64_t r1)
{
    const gram_arg *a = (const gram_arg *)p;
    const int R = a->R;
    for (int64_t n = 0; n < a->rows; ++n) {
        const double *f = a->F + n * R;
        for (int64_t r = r0; r < r1; ++r)
            for (int s = 0; s < R; ++s)
                a->G[r * R + s] += f[r] * f[s];
    }
}

static void gram(int64_t rows, int R, const double *F, double *G)
{
    memset(G, 0, sizeof(double) * (size_t)R * R);
    gram_arg a = {rows, R, F, G};
    if (g_threads > 1 && rows * R > 65536) par_for(R, gram_part, &a);
    else gram_part(&a, 0, R);
}

/* Cholesky H = L L^T (L lower, row-major).  Returns 0 on success, -1 when a
 * pivot falls to or below R * eps * max(diag H): H is then treated as
 * singular and the caller switches to the pseudo-inverse. */
static int cholesky(int R, const double *H, double *L)
{
    double dmax = 0.0;
    for (int r = 0; r < R; ++r)
        if (H[r * R + r] > dmax) dmax = H[r * R + r];
    const double tol = (double)R * DBL_EPSILON * dmax;
    if (!(dmax > 0.0)) return -1;
    memset(L, 0, sizeof(double) * (size_t)R * R);
    for (int j = 0; j < R; ++j) {
        double d = H[j * R + j];
        for (int k = 0; k < j; ++k) d -= L[j * R + k] * L[j * R + k];
        if (!(d > tol)) return -1;
        const double ljj = sqrt(d);
        L[j * R + j] = ljj;
        for (int i = j + 1; i < R; ++i) {
            double s = H[i * R + j];
            for (int k = 0; k < j; ++k) s -= L[i * R + k] * L[j * R + k];
            L[i * R + j] = s / ljj;
        }
    }
    return 0;
}

/* Cyclic Jacobi eigen-decomposition of symmetric H: H = V diag(w) V^T.
 * V is row-major with eigenvectors in columns. */
static void jacobi_eigen(int R, const double *H, double *w, double *V)
{
    double *A = (double *)malloc(sizeof(double) * (size_t)R * R);
    memcpy(A, H, sizeof(double) * (size_t)R * R);
    for (int i = 0; i < R; ++i)
        for (int j = 0; j < R; ++j) V[i * R + j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < R; ++i)
            for (int j = 0; j < R; ++j) {
                tot += A[i * R + j] * A[i * R + j];
                if (i != j) off += A[i * R + j] * A[i * R + j];
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int p = 0; p < R - 1; ++p)
            for (int q = p + 1; q < R; ++q) {
                const double apq = A[p * R + q];
                if (apq == 0.0) continue;
                const double app = A[p * R + p], aqq = A[q * R + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) /
                                 (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                /* A <- J^T A J with the rotation in the (p, q) plane */
                for (int k = 0; k < R; ++k) {
                    const double akp = A[k * R + p], akq = A[k * R + q];
                    A[k * R + p] = c * akp - s * akq;
                    A[k * R + q] = s * akp + c * akq;
                }
                for (int k = 0; k < R; ++k) {
                    const double apk = A[p * R + k], aqk = A[q * R + k];
                    A[p * R + k] = c * apk - s * aqk;
                    A[q * R + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < R; ++k) {
                    const double vkp = V[k * R + p], vkq = V[k * R + q];
                    V[k * R + p] = c * vkp - s * vkq;
                    V[k * R + q] = s * vkp + c * vkq;
                }
            }
    }
    for (int i = 0; i < R; ++i) w[i] = A[i * R + i];
    free(A);
}

/* Moore-Penrose pseudo-inverse of symmetric PSD H via its eigen-
 * decomposition; eigenvalues at or below R * eps * max eigenvalue are
 * treated as zero. */
static void pinv_sym(int R, const double *H, double *P)
{
    double *w = (double *)malloc(sizeof(double) * (size_t)R);
    double *V = (double *)malloc(sizeof(double) * (size_t)R * R);
    jacobi_eigen(R, H, w, V);
    double wmax = 0.0;
    for (int i = 0; i < R; ++i)
        if (w[i] > wmax) wmax = w[i];
    const double tol = (double)R * DBL_EPSILON * wmax;
    memset(P, 0, sizeof(double) * (size_t)R * R);
    for (int e = 0; e < R; ++e) {
        if (!(w[e] > tol)) continue;
        const double inv = 1.0 / w[e];
        for (int i = 0; i < R; ++i)
            for (int j = 0; j < R; ++j)
                P[i * R + j] += V[i * R + e] * inv * V[j * R + e];
    }
    free(w);
    free(V);
}

/* F <- M H^{-1} row by row (H symmetric).  Cholesky with forward and back
 * substitution; pseudo-inverse when H is numerically singular.  Rows are
 * independent (threads take disjoint row ranges).
 * Returns 0 if Cholesky was used, 1 if the pseudo-inverse was used. */
typedef struct {
    int R;
    const double *M, *L, *P; /* L: Cholesky factor, or P: pseudo-inverse */
    double *F;
} solve_arg;

static void solve_part(void *p, int64_t n0, int64_t n1)
{
    const solve_arg *a = (const solve_arg *)p;
    const int R = a->R;
    const double *L = a->L, *P = a->P;
    double *y = (double *)malloc(sizeof(double) * (size_t)R);
    for (int64_t n = n0; n < n1; ++n) {
        const double *m = a->M + n * R;
        double *x = a->F + n * R;
        if (L) {
            /* H x = m  with H = L L^T  (x is the row written as a column) */
            for (int i = 0; i < R; ++i) {
                double s = m[i];
                for (int k = 0; k < i; ++k) s -= L[i * R + k] * y[k];
                y[i] = s / L[i * R + i];
            }
            for (int i = R - 1; i >= 0; --i) {
                double s = y[i];
                for (int k = i + 1; k < R; ++k) s -= L[k * R + i] * x[k];
                x[i] = s / L[i * R + i];
            }
        } else {
            for (int s = 0; s < R; ++s) {
                double acc = 0.0;
                for (int r = 0; r < R; ++r) acc += m[r] * P[r * R + s];
                x[s] = acc;
            }
        }
    }
    free(y);
}

static int solve_rows(int64_t rows, int R, const double *M, const double *H,
                      double *F)
{
    double *L = (double *)malloc(sizeof(double) * (size_t)R * R);
    double *P = NULL;
    int used_pinv = 0;
    if (cholesky(R, H, L) != 0) {
        used_pinv = 1;
        P = (double *)malloc(sizeof(double) * (size_t)R * R);
        pinv_sym(R, H, P);
    }
    solve_arg a = {R, M, used_pinv ? NULL : L, P, F};
    if (g_threads > 1 && rows > 4096) par_for(rows, solve_part, &a);
    else solve_part(&a, 0, rows);
    free(P);
    free(L);
    return used_pinv;
}

/* ------------------------------------------------------------------ */
/* coordinate helpers                                                  */
/* ------------------------------------------------------------------ */

/* The three index arrays as one table: idx[m][e] is the mode-m index of
 * nonzero e (m = 0: i, 1: j, 2: k). */
typedef struct {
    const uint32_t *idx[3];
} coords;

/* Per mode n, the flattening that feeds it is ordered (root, mid, leaf):
 *   mode 0: (i, k, j)  -- fibers x_{i,:,k}, the rows of (X2)^T  (Lemma 1)
 *   mode 1: (j, i, k)  -- fibers x_{i,j,:}, the rows of (X3)^T
 *   mode 2: (k, j, i)  -- fibers x_{:,j,k}, the rows of (X1)^T
 * which are the three products used in Algorithm 4 (Appendix E).  With this
 * order the flattening of mode n is the CSR matrix X^{n+1} of eq. (1): row
 * = root, column = leaf + mid * dims[leaf]. */
static const int ROOT[3] = {0, 1, 2};
static const int MID[3] = {2, 0, 1};
static const int LEAF[3] = {1, 2, 0};

typedef struct {
    uint32_t key[3]; /* root, mid, leaf */
    double v;
    int64_t pos; /* original position, breaks ties so the sort is stable */
} rec;

static int rec_cmp(const void *a, const void *b)
{
    const rec *x = (const rec *)a, *y = (const rec *)b;
    for (int t = 0; t < 3; ++t) {
        if (x->key[t] < y->key[t]) return -1;
        if (x->key[t] > y->key[t]) return 1;
    }
    return (x->pos < y->pos) ? -1 : (x->pos > y->pos);
}

/* Sort nonzeros by (root, mid, leaf) of `mode` and sum duplicates in their
 * input order.  Returns a malloc'd array of distinct records and its size. */
static rec *sorted_distinct(int64_t nnz, coords c, const double *val, int mode,
                            int64_t *out_n)
{
    rec *a = (rec *)malloc(sizeof(rec) * (size_t)(nnz > 0 ? nnz : 1));
    for (int64_t e = 0; e < nnz; ++e) {
        a[e].key[0] = c.idx[ROOT[mode]][e];
        a[e].key[1] = c.idx[MID[mode]][e];
        a[e].key[2] = c.idx[LEAF[mode]][e];
        a[e].v = val[e];
        a[e].pos = e;
    }
    qsort(a, (size_t)nnz, sizeof(rec), rec_cmp);
    int64_t n = 0;
    for (int64_t e = 0; e < nnz; ++e) {
        if (n > 0 && a[n - 1].key[0] == a[e].key[0] &&
            a[n - 1].key[1] == a[e].key[1] && a[n - 1].key[2] == a[e].key[2]) {
            a[n - 1].v += a[e].v;
        } else {
            a[n++] = a[e];
        }
    }
    *out_n = n;
    return a;
}

/* ------------------------------------------------------------------ */
/* public entry points                                                  */
/* ------------------------------------------------------------------ */

/* MTTKRP by its element form (Lemma 2; Khatri-Rao definition, Appendix A):
 *   mode 0: out[i,:] += x_{ijk} * (B[j,:] * C[k,:])
 *   mode 1: out[j,:] += x_{ijk} * (A[i,:] * C[k,:])
 *   mode 2: out[k,:] += x_{ijk} * (A[i,:] * B[j,:])
 * F[m] is dims[m] x R row-major; out is dims[mode] x R and is overwritten. */
/* With threads: output rows are cut into g_threads ranges of about equal
 * nonzero counts; each thread adds the nonzeros of its rows in input order,
 * so every output row is the same sum in the same order as serially. */
typedef struct {
    int64_t nnz, rows;
    const uint32_t *root;   /* output-row index of each nonzero */
    const uint32_t *part;   /* row -> range (rows entries) */
    int T;                  /* ranges */
    uint32_t *hist;         /* per chunk: rows counts (pass 1), then T counts */
    int64_t *off;           /* per (chunk, range): first slot */
    uint32_t *order;        /* nonzero ids grouped by range, input order kept */
    /* the arithmetic */
    const uint32_t *ixp, *ixq;
    const double *val, *Fp, *Fq;
    int R;
    double *out;
} mtt_arg;

static void mtt_count_rows(void *p, int64_t c0, int64_t c1)
{
    mtt_arg *a = (mtt_arg *)p;
    for (int64_t c = c0; c < c1; ++c) {
        uint32_t *h = a->hist + c * a->rows;
        const int64_t e0 = a->nnz * c / a->T, e1 = a->nnz * (c + 1) / a->T;
        for (int64_t e = e0; e < e1; ++e) ++h[a->root[e]];
    }
}

static void mtt_count_parts(void *p, int64_t c0, int64_t c1)
{
    mtt_arg *a = (mtt_arg *)p;
    for (int64_t c = c0; c < c1; ++c) {
        int64_t *o = a->off + c * a->T;
        const int64_t e0 = a->nnz * c / a->T, e1 = a->nnz * (c + 1) / a->T;
        for (int64_t e = e0; e < e1; ++e) ++o[a->part[a->root[e]]];
    }
}

static void mtt_scatter(void *p, int64_t c0, int64_t c1)
{
    mtt_arg *a = (mtt_arg *)p;
    for (int64_t c = c0; c < c1; ++c) {
        int64_t *o = a->off + c * a->T;
        const int64_t e0 = a->nnz * c / a->T, e1 = a->nnz * (c + 1) / a->T;
        for (int64_t e = e0; e < e1; ++e) a->order[o[a->part[a->root[e]]]++] = (uint32_t)e;
    }
}

static void mtt_compute(void *p, int64_t t0, int64_t t1)
{
    mtt_arg *a = (mtt_arg *)p;
    const int R = a->R;
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t b = t == 0 ? 0 : a->off[(int64_t)(a->T - 1) * a->T + t - 1];
        const int64_t e1 = a->off[(int64_t)(a->T - 1) * a->T + t];
        for (int64_t x = b; x < e1; ++x) {
            const int64_t e = a->order[x];
            double *o = a->out + (int64_t)a->root[e] * R;
            const double *fp = a->Fp + (int64_t)a->ixp[e] * R;
            const double *fq = a->Fq + (int64_t)a->ixq[e] * R;
            for (int r = 0; r < R; ++r) o[r] += a->val[e] * fp[r] * fq[r];
        }
    }
}

void oracle_mttkrp(int64_t nnz, const uint32_t *i, const uint32_t *j,
                   const uint32_t *k, const double *val, const int64_t *dims,
                   int R, const double *A, const double *B, const double *C,
                   int mode, double *out)
{
    const uint32_t *ix[3] = {i, j, k};
    const double *F[3] = {A, B, C};
    const int p = (mode + 1) % 3, q = (mode + 2) % 3;
    memset(out, 0, sizeof(double) * (size_t)dims[mode] * R);
    const int T = g_threads;
    if (T <= 1 || nnz < 65536 || nnz > 0xFFFFFFFFll) {
        for (int64_t e = 0; e < nnz; ++e) {
            double *o = out + (int64_t)ix[mode][e] * R;
            const double *fp = F[p] + (int64_t)ix[p][e] * R;
            const double *fq = F[q] + (int64_t)ix[q][e] * R;
            for (int r = 0; r < R; ++r) o[r] += val[e] * fp[r] * fq[r];
        }
        return;
    }
    const int64_t rows = dims[mode];
    mtt_arg a;
    memset(&a, 0, sizeof(a));
    a.nnz = nnz;
    a.rows = rows;
    a.root = ix[mode];
    a.T = T;
    a.ixp = ix[p];
    a.ixq = ix[q];
    a.val = val;
    a.Fp = F[p];
    a.Fq = F[q];
    a.R = R;
    a.out = out;
    /* nonzeros per row (one histogram per input chunk, then summed) */
    a.hist = (uint32_t *)calloc((size_t)T * rows, sizeof(uint32_t));
    par_for(T, mtt_count_rows, &a);
    /* row ranges of about nnz / T nonzeros each */
    uint32_t *part = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)rows);
    int64_t acc = 0;
    int cur = 0;
    for (int64_t r = 0; r < rows; ++r) {
        int64_t c = 0;
        for (int t = 0; t < T; ++t) c += a.hist[(int64_t)t * rows + r];
        while (cur < T - 1 && acc >= nnz * (cur + 1) / T) ++cur;
        part[r] = (uint32_t)cur;
        acc += c;
    }
    free(a.hist);
    a.hist = NULL;
    a.part = part;
    /* per (chunk, range) counts -> first slots: range-major, chunk-minor,
     * so each range lists its nonzeros in input order */
    a.off = (int64_t *)calloc((size_t)T * T, sizeof(int64_t));
    par_for(T, mtt_count_parts, &a);
    int64_t run = 0;
    for (int t = 0; t < T; ++t)
        for (int c = 0; c < T; ++c) {
            const int64_t n = a.off[(int64_t)c * T + t];
            a.off[(int64_t)c * T + t] = run;
            run += n;
        }
    a.order = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)nnz);
    par_for(T, mtt_scatter, &a);
    /* after the scatter, off[(T-1) * T + t] is the end of range t */
    par_for(T, mtt_compute, &a);
    free(a.order);
    free(a.off);
    free(part);
}

/* Flattening of `mode` (Section 2.1 and the CSR discussion of Section 3):
 * distinct nonzeros sorted by (root, mid, leaf), duplicates summed.
 * Outputs (caller-allocated, sized for nnz entries):
 *   root_id[nroot], root_ptr[nroot+1] (fiber offsets),
 *   fib_mid[nfib], fib_ptr[nfib+1] (nonzero offsets), leaf[n], v[n].
 * Returns the number n of distinct nonzeros; *nroot and *nfib are set. */
int64_t oracle_flatten(int64_t nnz, const uint32_t *i, const uint32_t *j,
                       const uint32_t *k, const double *val, int mode,
                       uint32_t *root_id, int64_t *root_ptr, uint32_t *fib_mid,
                       int64_t *fib_ptr, uint32_t *leaf, double *v,
                       int64_t *nroot, int64_t *nfib)
{
    coords c = {{i, j, k}};
    int64_t n = 0;
    rec *a = sorted_distinct(nnz, c, val, mode, &n);
    int64_t nr = 0, nf = 0;
    for (int64_t e = 0; e < n; ++e) {
        const int new_root = (e == 0) || a[e].key[0] != a[e - 1].key[0];
        const int new_fib = new_root || a[e].key[1] != a[e - 1].key[1];
        if (new_root) {
            root_id[nr] = a[e].key[0];
            root_ptr[nr] = nf;
            ++nr;
        }
        if (new_fib) {
            fib_mid[nf] = a[e].key[1];
            fib_ptr[nf] = e;
            ++nf;
        }
        leaf[e] = a[e].key[2];
        v[e] = a[e].v;
    }
    root_ptr[nr] = nf;
    fib_ptr[nf] = n;
    *nroot = nr;
    *nfib = nf;
    free(a);
    return n;
}

/* First stage of Algorithm 1 for all R columns at once: for every nonempty
 * fiber f = (root, mid) of `mode`,
 *   P[f, r] = sum_{leaf} x * Fleaf[leaf, r],
 * i.e. the value arrays of the matrices M^r of Lemma 4 (for mode 0,
 * M^r[i, k] = sum_j x_{ijk} b_{jr}).  Fibers are in (root, mid) order, as
 * produced by oracle_flatten.  Returns the fiber count. */
int64_t oracle_fiber_partials(int64_t nnz, const uint32_t *i, const uint32_t *j,
                              const uint32_t *k, const double *val, int mode,
                              int R, const double *Fleaf, double *P)
{
    coords c = {{i, j, k}};
    int64_t n = 0;
    rec *a = sorted_distinct(nnz, c, val, mode, &n);
    int64_t nf = -1;
    for (int64_t e = 0; e < n; ++e) {
        const int new_fib = (e == 0) || a[e].key[0] != a[e - 1].key[0] ||
                            a[e].key[1] != a[e - 1].key[1];
        if (new_fib) {
            ++nf;
            for (int r = 0; r < R; ++r) P[nf * R + r] = 0.0;
        }
        for (int r = 0; r < R; ++r)
            P[nf * R + r] += a[e].v * Fleaf[(int64_t)a[e].key[2] * R + r];
    }
    free(a);
    return nf + 1;
}

/* Sum of squares of the distinct (duplicate-summed) entries, ||X||^2. */
double oracle_normsq(int64_t nnz, const uint32_t *i, const uint32_t *j,
                     const uint32_t *k, const double *val)
{
    if (g_distinct) { /* nothing to merge: the values in input order */
        double s = 0.0;
        for (int64_t e = 0; e < nnz; ++e) s += val[e] * val[e];
        return s;
    }
    coords c = {{i, j, k}};
    int64_t n = 0;
    rec *a = sorted_distinct(nnz, c, val, 0, &n);
    double s = 0.0;
    for (int64_t e = 0; e < n; ++e) s += a[e].v * a[e].v;
    free(a);
    return s;
}

/* <X, [[lambda; A, B, C]]> summed over the nonzeros directly:
 *   sum_e x_e sum_r lambda_r a_{ir} b_{jr} c_{kr}   (lambda NULL = ones). */
typedef struct {
    const uint32_t *i, *j, *k;
    int R;
    const double *A, *B, *C, *lambda;
    double *t;
} inner_arg;

static void inner_terms(void *p, int64_t e0, int64_t e1)
{
    const inner_arg *a = (const inner_arg *)p;
    const int R = a->R;
    for (int64_t e = e0; e < e1; ++e) {
        const double *x = a->A + (int64_t)a->i[e] * R;
        const double *y = a->B + (int64_t)a->j[e] * R;
        const double *z = a->C + (int64_t)a->k[e] * R;
        double t = 0.0;
        for (int r = 0; r < R; ++r)
            t += (a->lambda ? a->lambda[r] : 1.0) * x[r] * y[r] * z[r];
        a->t[e] = t;
    }
}

double oracle_inner(int64_t nnz, const uint32_t *i, const uint32_t *j,
                    const uint32_t *k, const double *val, int R,
                    const double *A, const double *B, const double *C,
                    const double *lambda)
{
    /* each nonzero's model value (threads: disjoint nonzeros), then the sum
     * over the nonzeros in input order */
    double *t = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    inner_arg a = {i, j, k, R, A, B, C, lambda, t};
    if (g_threads > 1 && nnz > 65536) par_for(nnz, inner_terms, &a);
    else inner_terms(&a, 0, nnz);
    double s = 0.0;
    for (int64_t e = 0; e < nnz; ++e) s += val[e] * t[e];
    free(t);
    return s;
}

/* One CP-ALS iteration (Algorithm 2 / Algorithm 4) in Gauss-Seidel order
 * n = 0, 1, 2, each step using the factors already updated:
 *   M   = MTTKRP(n)
 *   H   = (F_p^T F_p) * (F_q^T F_q) + reg I        (Appendix A identity)
 *   F_n = M H^{-1}  (Cholesky; pseudo-inverse when H is singular)
 *   lambda_r = ||F_n[:, r]||_2 ; F_n[:, r] /= lambda_r when lambda_r > 0.
 * After mode 2 the fit of the weighted model [[lambda; A, B, C]]:
 *   ||Xhat||^2 = lambda^T (G_A * G_B * G_C) lambda
 *   <X, Xhat>  = sum_r lambda_r sum_k C[k, r] M3[k, r]
 *   fit = 1 - sqrt(max(0, ||X||^2 + ||Xhat||^2 - 2 <X, Xhat>)) / ||X||
 *   (fit = 0 when ||X|| = 0).
 * store_bf16 != 0 models factors kept in BF16 storage: each new F_n is
 * rounded (FP32 then BF16, nearest-even) before the next mode uses it and
 * before the fit is formed; lambda comes from the unrounded F_n.
 * A, B, C are updated in place.  out[0] = fit, out[1] = <X,Xhat> computed
 * directly over the nonzeros (independent cross-check), out[2] = ||X||^2,
 * out[3] = ||Xhat||^2.  Returns a bitmask of the modes that used the
 * pseudo-inverse. */
/* Storage rounding of a factor entry kept in BF16: to the nearest FP32, then
 * to the nearest BF16 (round to nearest, ties to even on the FP32 bits). */
static double round_bf16(double x)
{
    float f = (float)x;
    uint32_t b;
    memcpy(&b, &f, 4);
    if ((b & 0x7F800000u) == 0x7F800000u) {
        b = (b & 0xFFFF0000u) | ((b & 0xFFFFu) ? 0x00400000u : 0u);
    } else {
        b += 0x7FFFu + ((b >> 16) & 1u);
        b &= 0xFFFF0000u;
    }
    memcpy(&f, &b, 4);
    return (double)f;
}

/* column pieces of the ALS step, split over columns r (each a sum over the
 * rows in order) or over entries */
typedef struct {
    int64_t rows;
    int R;
    double *F, *lambda;
} colnorm_arg;

static void colnorm_part(void *p, int64_t r0, int64_t r1)
{
    const colnorm_arg *a = (const colnorm_arg *)p;
    const int R = a->R;
    for (int64_t r = r0; r < r1; ++r) {
        double s = 0.0;
        for (int64_t m = 0; m < a->rows; ++m) s += a->F[m * R + r] * a->F[m * R + r];
        a->lambda[r] = sqrt(s);
        if (a->lambda[r] > 0.0)
            for (int64_t m = 0; m < a->rows; ++m) a->F[m * R + r] /= a->lambda[r];
    }
}

static void round_part(void *p, int64_t e0, int64_t e1)
{
    double *F = (double *)p;
    for (int64_t e = e0; e < e1; ++e) F[e] = round_bf16(F[e]);
}

typedef struct {
    int64_t rows;
    int R;
    const double *C, *M;
    double *out;
} coldot_arg;

static void coldot_part(void *p, int64_t r0, int64_t r1)
{
    const coldot_arg *a = (const coldot_arg *)p;
    const int R = a->R;
    for (int64_t r = r0; r < r1; ++r) {
        double s = 0.0;
        for (int64_t m = 0; m < a->rows; ++m) s += a->C[m * R + r] * a->M[m * R + r];
        a->out[r] = s;
    }
}

int oracle_als_iter(int64_t nnz, const uint32_t *i, const uint32_t *j,
                    const uint32_t *k, const double *val, const int64_t *dims,
                    int R, double reg, int store_bf16, double *A, double *B,
                    double *C, double *lambda, double *out)
{
    double *F[3] = {A, B, C};
    int64_t dmax = dims[0];
    if (dims[1] > dmax) dmax = dims[1];
    if (dims[2] > dmax) dmax = dims[2];
    double *M = (double *)malloc(sizeof(double) * (size_t)dmax * R);
    double *M3 = (double *)malloc(sizeof(double) * (size_t)dims[2] * R);
    double *Gp = (double *)malloc(sizeof(double) * (size_t)R * R);
    double *Gq = (double *)malloc(sizeof(double) * (size_t)R * R);
    double *H = (double *)malloc(sizeof(double) * (size_t)R * R);
    int pinv_mask = 0;
    for (int n = 0; n < 3; ++n) {
        const int p = (n + 1) % 3, q = (n + 2) % 3;
        oracle_mttkrp(nnz, i, j, k, val, dims, R, F[0], F[1], F[2], n, M);
        gram(dims[p], R, F[p], Gp);
        gram(dims[q], R, F[q], Gq);
        for (int t = 0; t < R * R; ++t) H[t] = Gp[t] * Gq[t];
        for (int r = 0; r < R; ++r) H[r * R + r] += reg;
        if (solve_rows(dims[n], R, M, H, F[n])) pinv_mask |= 1 << n;
        /* lambda_r = ||F_n[:, r]||_2, then unit columns (threads: columns) */
        colnorm_arg cn = {dims[n], R, F[n], lambda};
        if (g_threads > 1 && dims[n] > 4096) par_for(R, colnorm_part, &cn);
        else colnorm_part(&cn, 0, R);
        /* a factor stored in BF16 enters the next mode's update rounded */
        if (store_bf16) {
            if (g_threads > 1 && dims[n] > 4096) par_for(dims[n] * R, round_part, F[n]);
            else round_part(F[n], 0, dims[n] * R);
        }
        if (n == 2) memcpy(M3, M, sizeof(double) * (size_t)dims[2] * R);
    }
    /* fit */
    double *GA = (double *)malloc(sizeof(double) * (size_t)R * R);
    double *GB = (double *)malloc(sizeof(double) * (size_t)R * R);
    double *GC = (double *)malloc(sizeof(double) * (size_t)R * R);
    gram(dims[0], R, A, GA);
    gram(dims[1], R, B, GB);
    gram(dims[2], R, C, GC);
    double xhat2 = 0.0;
    for (int r = 0; r < R; ++r)
        for (int s = 0; s < R; ++s)
            xhat2 += lambda[r] * lambda[s] * GA[r * R + s] * GB[r * R + s] *
                     GC[r * R + s];
    /* <X, Xhat> = sum_r lambda_r sum_k C[k, r] M3[k, r] (threads: columns) */
    double *colsum = (double *)malloc(sizeof(double) * (size_t)R);
    coldot_arg cd = {dims[2], R, C, M3, colsum};
    if (g_threads > 1 && dims[2] > 4096) par_for(R, coldot_part, &cd);
    else coldot_part(&cd, 0, R);
    double inner = 0.0;
    for (int r = 0; r < R; ++r) inner += lambda[r] * colsum[r];
    free(colsum);
    const double x2 = oracle_normsq(nnz, i, j, k, val);
    double res2 = x2 + xhat2 - 2.0 * inner;
    if (res2 < 0.0) res2 = 0.0;
    out[0] = (x2 > 0.0) ? 1.0 - sqrt(res2) / sqrt(x2) : 0.0;
    out[1] = oracle_inner(nnz, i, j, k, val, R, A, B, C, lambda);
    out[2] = x2;
    out[3] = xhat2;
    free(GA);
    free(GB);
    free(GC);
    free(M);
    free(M3);
    free(Gp);
    free(Gq);
    free(H);
    return pinv_mask;
}

/* GD gradient (Appendix C; Algorithm 3 with the minus sign of the gradient
 * equation), all three at the same point, unit weights:
 *   grad_n = -MTTKRP(n) + F_n ((F_p^T F_p) * (F_q^T F_q) + reg I)
 *   f = 1/2 (||X||^2 - 2 <X, [[A,B,C]]> + sum(G_A * G_B * G_C))
 *       + 1/2 reg (||A||^2 + ||B||^2 + ||C||^2)
 * The sum in f runs over every (i, j, k), so zeros count.  G[m] receives a
 * dims[m] x R gradient.  Returns f. */
/* gradient rows g = -M + F H (threads: rows) */
typedef struct {
    int R;
    const double *F, *H;
    double *G;
} gdrow_arg;

static void gdrow_part(void *p, int64_t m0, int64_t m1)
{
    const gdrow_arg *a = (const gdrow_arg *)p;
    const int R = a->R;
    for (int64_t m = m0; m < m1; ++m) {
        const double *fr = a->F + m * R;
        double *g = a->G + m * R;
        for (int s = 0; s < R; ++s) {
            double acc = 0.0;
            for (int r = 0; r < R; ++r) acc += fr[r] * a->H[r * R + s];
            g[s] = -g[s] + acc;
        }
    }
}

double oracle_gd_grad(int64_t nnz, const uint32_t *i, const uint32_t *j,
                      const uint32_t *k, const double *val,
                      const int64_t *dims, int R, double reg, const double *A,
                      const double *B, const double *C, double *GA_out,
                      double *GB_out, double *GC_out)
{
    const double *F[3] = {A, B, C};
    double *Gout[3] = {GA_out, GB_out, GC_out};
    double *Gm[3];
    for (int m = 0; m < 3; ++m) {
        Gm[m] = (double *)malloc(sizeof(double) * (size_t)R * R);
        gram(dims[m], R, F[m], Gm[m]);
    }
    double *H = (double *)malloc(sizeof(double) * (size_t)R * R);
    for (int n = 0; n < 3; ++n) {
        const int p = (n + 1) % 3, q = (n + 2) % 3;
        oracle_mttkrp(nnz, i, j, k, val, dims, R, A, B, C, n, Gout[n]);
        for (int t = 0; t < R * R; ++t) H[t] = Gm[p][t] * Gm[q][t];
        for (int r = 0; r < R; ++r) H[r * R + r] += reg;
        gdrow_arg ga = {R, F[n], H, Gout[n]};
        if (g_threads > 1 && dims[n] > 4096) par_for(dims[n], gdrow_part, &ga);
        else gdrow_part(&ga, 0, dims[n]);
    }
    double xhat2 = 0.0, fro2 = 0.0;
    for (int t = 0; t < R * R; ++t) xhat2 += Gm[0][t] * Gm[1][t] * Gm[2][t];
    for (int m = 0; m < 3; ++m)
        for (int r = 0; r < R; ++r) fro2 += Gm[m][r * R + r];
    const double x2 = oracle_normsq(nnz, i, j, k, val);
    const double inner = oracle_inner(nnz, i, j, k, val, R, A, B, C, NULL);
    for (int m = 0; m < 3; ++m) free(Gm[m]);
    free(H);
    return 0.5 * (x2 - 2.0 * inner + xhat2) + 0.5 * reg * fro2;
}

/* GD objective at one point (Appendix C, unit weights), from its definition
 * through the identity ||[[A,B,C]]||^2 = sum(G_A * G_B * G_C) (Appendix A):
 *   f = 1/2 (||X||^2 - 2 <X, [[A,B,C]]> + ||[[A,B,C]]||^2)
 *       + 1/2 reg (||A||^2 + ||B||^2 + ||C||^2). */
double oracle_objective(int64_t nnz, const uint32_t *i, const uint32_t *j,
                        const uint32_t *k, const double *val, const int64_t *dims, int R,
                        double reg, const double *A, const double *B, const double *C)
{
    const double *F[3] = {A, B, C};
    double *Gm[3];
    for (int m = 0; m < 3; ++m) {
        Gm[m] = (double *)malloc(sizeof(double) * (size_t)R * R);
        gram(dims[m], R, F[m], Gm[m]);
    }
    double xhat2 = 0.0, fro2 = 0.0;
    for (int t = 0; t < R * R; ++t) xhat2 += Gm[0][t] * Gm[1][t] * Gm[2][t];
    for (int m = 0; m < 3; ++m)
        for (int r = 0; r < R; ++r) fro2 += Gm[m][r * R + r];
    for (int m = 0; m < 3; ++m) free(Gm[m]);
    const double x2 = oracle_normsq(nnz, i, j, k, val);
    const double inner = oracle_inner(nnz, i, j, k, val, R, A, B, C, NULL);
    return 0.5 * (x2 - 2.0 * inner + xhat2) + 0.5 * reg * fro2;
}

/* One full GD iteration of DFacTo (Algorithm 5 / Algorithm 3): the three
 * gradients at the same point (oracle_gd_grad), then a backtracking line
 * search, then the simultaneous update of A, B and C.  The paper names a
 * backtracking line search without its constants; here (Armijo): trial
 * steps alpha = alpha0 * shrink^t, t = 0 .. max_trials - 1, with trial
 * factors F_m - alpha grad_m (rounded to BF16 storage when store_bf16), and
 * the first trial with
 *   f(trial) <= f(F) - c * alpha * (||grad_A||^2 + ||grad_B||^2 + ||grad_C||^2)
 * is taken.  If no trial passes, the factors are left unchanged.
 * A, B, C are updated in place.  out[0] = f at the input, out[1] = f at the
 * returned factors, out[2] = the squared gradient norm, out[3] = the step
 * taken (0 if none), out[4] = trials evaluated.  Returns 1 if a step was
 * taken. */
int oracle_gd_step(int64_t nnz, const uint32_t *i, const uint32_t *j, const uint32_t *k,
                   const double *val, const int64_t *dims, int R, double reg, double *A,
                   double *B, double *C, double alpha0, double shrink, double c,
                   int max_trials, int store_bf16, double *out)
{
    double *F[3] = {A, B, C};
    double *G[3], *T[3];
    for (int m = 0; m < 3; ++m) {
        G[m] = (double *)malloc(sizeof(double) * (size_t)dims[m] * R);
        T[m] = (double *)malloc(sizeof(double) * (size_t)dims[m] * R);
    }
    const double f0 = oracle_gd_grad(nnz, i, j, k, val, dims, R, reg, A, B, C, G[0], G[1], G[2]);
    double g2 = 0.0;
    for (int m = 0; m < 3; ++m)
        for (int64_t e = 0; e < dims[m] * R; ++e) g2 += G[m][e] * G[m][e];
    double alpha = alpha0, f = f0;
    int trials = 0, taken = 0;
    for (int t = 0; t < max_trials; ++t) {
        for (int m = 0; m < 3; ++m)
            for (int64_t e = 0; e < dims[m] * R; ++e) {
                const double x = F[m][e] - alpha * G[m][e];
                T[m][e] = store_bf16 ? round_bf16(x) : x;
            }
        const double ft = oracle_objective(nnz, i, j, k, val, dims, R, reg, T[0], T[1], T[2]);
        ++trials;
        if (ft <= f0 - c * alpha * g2) {
            for (int m = 0; m < 3; ++m)
                memcpy(F[m], T[m], sizeof(double) * (size_t)dims[m] * R);
            f = ft;
            taken = 1;
            break;
        }
        alpha *= shrink;
    }
    for (int m = 0; m < 3; ++m) {
        free(G[m]);
        free(T[m]);
    }
    out[0] = f0;
    out[1] = f;
    out[2] = g2;
    out[3] = taken ? alpha : 0.0;
    out[4] = (double)trials;
    return taken;
}

/* ------------------------------------------------------------------ */
/* joint matrix completion and tensor factorization                     */
/* ------------------------------------------------------------------ */

/* The joint model (the section on joint matrix completion and tensor
 * factorization): a ratings matrix Y (users x items, observed entries
 * (yi[e], yj[e]) -> yv[e]) shares the user factor A and the item factor B
 * with the user x item x word tensor X:
 *   f = 1/2 sum_{(i,j) observed} (y_ij - a_i . b_j)^2
 *       + mu 1/2 sum_{i,j,k} (x_ijk - [[A,B,C]]_ijk)^2
 *       + lam 1/2 (||A||^2 + ||B||^2 + ||C||^2)
 * (the tensor sum runs over every cell, as in the GD objective).
 * Gradient rows (the paper's per-row gradient eq.; ridge lam):
 *   g_a_i = -sum_{j in row i} (y_ij - a_i.b_j) b_j + mu (-M0 + A H0)_i + lam a_i
 *   g_b_j = -sum_{i in col j} (y_ij - a_i.b_j) a_i + mu (-M1 + B H1)_j + lam b_j
 *   g_c_k =                                          mu (-M2 + C H2)_k + lam c_k
 * with M_n the MTTKRPs and H_n the Hadamard products of the other two
 * Grams.  Returns f. */
double oracle_joint_grad(int64_t nnz, const uint32_t *i, const uint32_t *j, const uint32_t *k,
                         const double *val, const int64_t *dims, int64_t ny,
                         const uint32_t *yi, const uint32_t *yj, const double *yv, int R,
                         double mu, double lam, const double *A, const double *B,
                         const double *C, double *gA, double *gB, double *gC)
{
    const double *F[3] = {A, B, C};
    double *Gout[3] = {gA, gB, gC};
    double *Gm[3];
    for (int m = 0; m < 3; ++m) {
        Gm[m] = (double *)malloc(sizeof(double) * (size_t)R * R);
        gram(dims[m], R, F[m], Gm[m]);
    }
    double *H = (double *)malloc(sizeof(double) * (size_t)R * R);
    for (int n = 0; n < 3; ++n) {
        const int p = (n + 1) % 3, q = (n + 2) % 3;
        oracle_mttkrp(nnz, i, j, k, val, dims, R, A, B, C, n, Gout[n]);
        for (int t = 0; t < R * R; ++t) H[t] = Gm[p][t] * Gm[q][t];
        for (int64_t m = 0; m < dims[n]; ++m) {
            const double *fr = F[n] + m * R;
            double *g = Gout[n] + m * R;
            for (int s = 0; s < R; ++s) {
                double acc = 0.0;
                for (int r = 0; r < R; ++r) acc += fr[r] * H[r * R + s];
                g[s] = mu * (-g[s] + acc) + lam * fr[s];
            }
        }
    }
    double fy = 0.0;
    for (int64_t e = 0; e < ny; ++e) {
        const double *a = A + (int64_t)yi[e] * R, *b = B + (int64_t)yj[e] * R;
        double dot = 0.0;
        for (int r = 0; r < R; ++r) dot += a[r] * b[r];
        const double res = yv[e] - dot;
        fy += 0.5 * res * res;
        double *ga = gA + (int64_t)yi[e] * R, *gb = gB + (int64_t)yj[e] * R;
        for (int r = 0; r < R; ++r) {
            ga[r] -= res * b[r];
            gb[r] -= res * a[r];
        }
    }
    double xhat2 = 0.0, fro2 = 0.0;
    for (int t = 0; t < R * R; ++t) xhat2 += Gm[0][t] * Gm[1][t] * Gm[2][t];
    for (int m = 0; m < 3; ++m)
        for (int r = 0; r < R; ++r) fro2 += Gm[m][r * R + r];
    const double x2 = oracle_normsq(nnz, i, j, k, val);
    const double inner = oracle_inner(nnz, i, j, k, val, R, A, B, C, NULL);
    for (int m = 0; m < 3; ++m) free(Gm[m]);
    free(H);
    return fy + mu * 0.5 * (x2 - 2.0 * inner + xhat2) + 0.5 * lam * fro2;
}

/* One ALS iteration of the joint model in the order A, B, C (Gauss-Seidel),
 * each row set to the minimizer of f with the other factors fixed (the
 * paper's closed form, from its per-row gradient set to zero):
 *   a_i = (sum_{j in row i} y_ij b_j + mu M0_i)
 *         (sum_{j in row i} b_j^T b_j + mu (B^T B * C^T C) + lam I)^{-1}
 * and likewise for b_j over the users who rated item j (with A^T A * C^T C);
 * c_k = mu M2_k (mu (A^T A * B^T B) + lam I)^{-1} (no ratings term).  Each
 * R x R system is solved by Cholesky, or the pseudo-inverse when it is
 * numerically singular.  store_bf16 != 0 models factors kept in BF16
 * storage: each new factor is rounded to BF16 before later use.  A, B, C are
 * updated in place; returns f at the new point. */
/* Row `row` of mode n's block of the joint ALS (the closed form above):
 * S = mu (Gp * Gq) + lam I + sum over the row's ratings of v v^T, rhs =
 * mu M[row] + sum y v, with v the other side's factor row (n < 2; the words
 * mode has no ratings term); out = S^-1 rhs.  S and rhs are scratch. */
static void joint_row(int n, int64_t row, int R, double mu, double lam, const double *Gp,
                      const double *Gq, const double *M, int64_t ny, const uint32_t *own,
                      const uint32_t *other, const double *yv, const double *Fo, double *S,
                      double *rhs, double *out)
{
    for (int t = 0; t < R * R; ++t) S[t] = mu * Gp[t] * Gq[t];
    for (int r = 0; r < R; ++r) {
        S[r * R + r] += lam;
        rhs[r] = mu * M[row * R + r];
    }
    if (n < 2) {  /* the ratings of this user (n = 0) or item (n = 1) */
        for (int64_t e = 0; e < ny; ++e) {
            if ((int64_t)own[e] != row) continue;
            const double *v = Fo + (int64_t)other[e] * R;
            for (int r = 0; r < R; ++r) {
                rhs[r] += yv[e] * v[r];
                for (int s = 0; s < R; ++s) S[r * R + s] += v[r] * v[s];
            }
        }
    }
    solve_rows(1, R, rhs, S, out);
}

double oracle_joint_als_iter(int64_t nnz, const uint32_t *i, const uint32_t *j,
                             const uint32_t *k, const double *val, const int64_t *dims,
                             int64_t ny, const uint32_t *yi, const uint32_t *yj,
                             const double *yv, int R, double mu, double lam, int store_bf16,
                             double *A, double *B, double *C)
{
    double *F[3] = {A, B, C};
    const uint32_t *own[2] = {yi, yj}, *other[2] = {yj, yi};
    double *Gp = (double *)malloc(sizeof(double) * (size_t)R * R);
    double *Gq = (double *)malloc(sizeof(double) * (size_t)R * R);
    double *S = (double *)malloc(sizeof(double) * (size_t)R * R);
    double *rhs = (double *)malloc(sizeof(double) * (size_t)R);
    for (int n = 0; n < 3; ++n) {
        const int p = (n + 1) % 3, q = (n + 2) % 3;
        double *M = (double *)malloc(sizeof(double) * (size_t)dims[n] * R);
        oracle_mttkrp(nnz, i, j, k, val, dims, R, A, B, C, n, M);
        gram(dims[p], R, F[p], Gp);
        gram(dims[q], R, F[q], Gq);
        for (int64_t row = 0; row < dims[n]; ++row)
            joint_row(n, row, R, mu, lam, Gp, Gq, M, ny, n < 2 ? own[n] : NULL,
                      n < 2 ? other[n] : NULL, yv, n < 2 ? F[1 - n] : NULL, S, rhs,
                      F[n] + row * R);
        if (store_bf16)
            for (int64_t e = 0; e < dims[n] * R; ++e) F[n][e] = round_bf16(F[n][e]);
        free(M);
    }
    free(Gp);
    free(Gq);
    free(S);
    free(rhs);
    double *g[3];
    for (int m = 0; m < 3; ++m) g[m] = (double *)malloc(sizeof(double) * (size_t)dims[m] * R);
    const double f = oracle_joint_grad(nnz, i, j, k, val, dims, ny, yi, yj, yv, R, mu, lam, A, B,
                                       C, g[0], g[1], g[2]);
    for (int m = 0; m < 3; ++m) free(g[m]);
    return f;
}

/* The listed rows of mode n's block (n = 0 users, 1 items) of one joint ALS
 * iteration, from the factors as given (A, B, C: for n = 1 pass the updated
 * A), each as in oracle_joint_als_iter: out[q] = row rows[q] (nrows x R).
 * For checking sampled rows of a large problem: only the listed rows are
 * solved. */
void oracle_joint_als_rows(int64_t nnz, const uint32_t *i, const uint32_t *j, const uint32_t *k,
                           const double *val, const int64_t *dims, int64_t ny,
                           const uint32_t *yi, const uint32_t *yj, const double *yv, int R,
                           double mu, double lam, const double *A, const double *B,
                           const double *C, int n, int64_t nrows, const int64_t *rows,
                           double *out)
{
    const double *F[3] = {A, B, C};
    const int p = (n + 1) % 3, q = (n + 2) % 3;
    double *Gp = (double *)malloc(sizeof(double) * (size_t)R * R);
    double *Gq = (double *)malloc(sizeof(double) * (size_t)R * R);
    double *S = (double *)malloc(sizeof(double) * (size_t)R * R);
    double *rhs = (double *)malloc(sizeof(double) * (size_t)R);
    double *M = (double *)malloc(sizeof(double) * (size_t)dims[n] * R);
    oracle_mttkrp(nnz, i, j, k, val, dims, R, A, B, C, n, M);
    gram(dims[p], R, F[p], Gp);
    gram(dims[q], R, F[q], Gq);
    for (int64_t t = 0; t < nrows; ++t)
        joint_row(n, rows[t], R, mu, lam, Gp, Gq, M, ny, n == 0 ? yi : yj, n == 0 ? yj : yi, yv,
                  F[1 - n], S, rhs, out + t * R);
    free(M);
    free(Gp);
    free(Gq);
    free(S);
    free(rhs);
}
