// group.hip -- grouped CP-ALS over many independent tensors (batched solves).
//
// Each step of an ALS iteration (Algorithm 2 / Algorithm 4 per member) is
// enqueued as one launch per kernel class for all members together: the
// MTTKRP as a persistent grid walking a work list of (tensor, chunk group)
// items, the carry fix-ups over combined run tables, and the small dense
// steps (Grams, solve, lambda and fit, row map) over tables of (tensor,
// block) pairs.  Per member the arithmetic, the work split and the order of
// every reduction are those of dfacto_als_iter, so the results are bitwise
// the same as running the members one by one.  One iteration can be captured
// once as a HIP graph and replayed.  A small autotuner picks the launch form
// of each MTTKRP kernel class (persistent grid size, columns per lane, chunks
// per lane group) by timing candidates on the group's
// own data (none of these choices changes any result).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <tuple>
#include <vector>

#include "internal.hpp"

namespace {
using namespace dfacto;

// Ranks with a grouped row map (LDS-tiled or matrix-core kernels).
bool group_rank_ok(int R) {
    return R == 4 || R == 8 || R == 12 || R == 16 || R == 32 || R == 48 || R == 64;
}
}  // namespace

struct dfacto_group {
    int device = 0;
    int n = 0, maxR = 0;
    dfacto_dtype dtype = DFACTO_F32;
    dfacto_ctx gctx;  // bound to the group's own stream; no workspace use
    hipStream_t stream = nullptr;
    bool own_stream = true;  // false: launches go to the creating context's stream
    DevMem mem;  // the creating context's memory source
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::vector<void *> allocs;
    size_t bytes = 0;
    std::vector<std::function<void()>> steps;  // enqueue one iteration
    int launches = 0;                          // kernel launches per iteration
    bool use_graph = false;
    // Captured iterations: [0] every step, [1] from open_end on (see below)
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    // BF16 storage: an iteration opens with the Grams of the stored B and C,
    // which are exactly the Grams the previous iteration formed last for
    // those factors (same kernels, same data).  Iterations after the first
    // of a call -- and, with DFACTO_GROUP_OWN_FACTORS, after the group's
    // previous iteration -- start at open_end instead.
    size_t open_end = 0;
    bool reuse_grams = false;   // BF16 storage
    bool own_factors = false;   // DFACTO_GROUP_OWN_FACTORS
    bool grams_valid = false;   // an iteration has run since creation
    // One grouped MTTKRP launch per kernel class and mode: its shape (columns
    // per lane, lanes per group), chunks per lane group, work items (one
    // table per item size) and persistent grid size.  The fix-ups after it
    // keep the class's own shape (the carries do not depend on the one the
    // MTTKRP ran with).  cands: the launch forms the tuner may choose.
    struct MtVariant {
        MttkrpShape sh;
        unsigned kper;
        const uint2 *items;
        uint32_t nitems;
    };
    struct MtLaunch {
        MtVariant v;
        bool small;
        unsigned grid;
        std::vector<MtVariant> cands;
    };
    std::vector<MtLaunch> mt;
    // Small tables built on the host go to arena chunks (device memory of at
    // least 4 MB) through one host staging buffer per chunk, copied once the
    // group is built (the staging stays until the group is freed, so the
    // copy is asynchronous).  Tables combined from the members' device lists
    // (work items, runs, empty rows) are expanded on the device into
    // separately reserved space.
    struct Chunk {
        char *dev;
        size_t cap, used;
        std::vector<char> host;
    };
    std::deque<Chunk> arena;
    char *dev_arena = nullptr;
    size_t dev_left = 0;
};

namespace {

// Stream-ordered allocations on the group's stream: creating and freeing a
// group never waits for unrelated work on the device.
template <typename T>
T *dev_alloc(dfacto_group *g, size_t count) {
    void *p = nullptr;
    const size_t bytes = std::max<size_t>(sizeof(T) * count, 256);
    hip_check(g->mem.alloc(&p, bytes, g->stream), "group allocation");
    g->allocs.push_back(p);
    g->bytes += bytes;
    return (T *)p;
}

// A host table's place in the arena; its bytes are staged and copied with
// the whole chunk by upload_all().
template <typename T>
T *upload(dfacto_group *g, const std::vector<T> &v) {
    const size_t bytes = (std::max<size_t>(v.size(), 1) * sizeof(T) + 255) & ~(size_t)255;
    if (g->arena.empty() || g->arena.back().cap - g->arena.back().used < bytes) {
        const size_t cap = std::max<size_t>(bytes, 4u << 20);
        g->arena.push_back({dev_alloc<char>(g, cap), cap, 0, {}});
    }
    dfacto_group::Chunk &c = g->arena.back();
    T *d = (T *)(c.dev + c.used);
    c.host.resize(c.used + bytes);
    if (!v.empty()) std::memcpy(c.host.data() + c.used, v.data(), sizeof(T) * v.size());
    c.used += bytes;
    return d;
}

void upload_all(dfacto_group *g) {
    for (dfacto_group::Chunk &c : g->arena)
        if (c.used)
            DF_HIP(hipMemcpyAsync(c.dev, c.host.data(), c.used, hipMemcpyHostToDevice, g->stream));
}

// Device space for an expanded table (chunks of at least 16 MB).
template <typename T>
T *dev_reserve(dfacto_group *g, size_t count) {
    const size_t bytes = (std::max<size_t>(count, 1) * sizeof(T) + 255) & ~(size_t)255;
    if (g->dev_left < bytes) {
        const size_t cap = std::max<size_t>(bytes, 16u << 20);
        g->dev_arena = dev_alloc<char>(g, cap);
        g->dev_left = cap;
    }
    T *d = (T *)g->dev_arena;
    g->dev_arena += bytes;
    g->dev_left -= bytes;
    return d;
}

// One member's part of a combined table: `count` elements from `off` on.
// width 0: (t, x * step) work items; 1: (t, src[x]); 3: (t, src[3x],
// src[3x + 1], src[3x + 2]).
struct ExpandJob {
    const uint32_t *src;
    uint64_t off;
    uint32_t t, count, width, step;
};

// out[x] for x < total from the job whose range holds x (jobs in order of off)
template <typename V>
__global__ __launch_bounds__(256) void k_expand(const ExpandJob *__restrict__ jobs, int njobs,
                                                uint64_t total, V *__restrict__ out) {
    for (uint64_t x = blockIdx.x * 256ull + threadIdx.x; x < total;
         x += (uint64_t)gridDim.x * 256ull) {
        int lo = 0, hi = njobs - 1;  // the last job with off <= x
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (jobs[mid].off <= x) lo = mid;
            else hi = mid - 1;
        }
        const ExpandJob j = jobs[lo];
        const uint32_t e = (uint32_t)(x - j.off);
        if constexpr (sizeof(V) == 8) {
            out[x] = make_uint2(j.t, j.width ? j.src[e] : e * j.step);
        } else {
            const uint32_t *p = j.src + 3ull * e;
            out[x] = make_uint4(j.t, p[0], p[1], p[2]);
        }
    }
}

// A combined table whose jobs are uploaded now and expanded after upload_all.
template <typename V>
struct Expansion {
    std::vector<ExpandJob> jobs;
    uint64_t total = 0;
    V *out = nullptr;
    void add(uint32_t t, const uint32_t *src, uint64_t count, uint32_t width, uint32_t step) {
        if (count == 0) return;
        jobs.push_back({src, total, t, (uint32_t)count, width, step});
        total += count;
    }
};

// Per-member device workspace.
struct MemberWs {
    float *M, *carry;
    void *perm;  // permuted tables of a relabeled member (else null)
    double *G[3], *Hinv, *W, *MtM, *solve_scratch, *lam_scratch, *part;
    int *flag;
};

struct Build {
    dfacto_group *g;
    const std::vector<const dfacto_tensor *> &T;
    const std::vector<int> &R;
    double reg;
    void *const *F;  // 3n
    double *const *lambda;
    double *fit;
    std::vector<MemberWs> ws;
    std::vector<std::function<void()>> mt_steps;  // the MTTKRP launches, for tuning
    std::vector<size_t> mt_index;                 // their entries in g->mt
    bool tuning = false;                          // build the tuner's launch forms
    std::vector<std::function<void()>> post;      // table expansions, after upload_all

    // device space for a combined table; its expansion runs after upload_all
    template <typename V>
    V *expand(const Expansion<V> &x) {
        V *out = dev_reserve<V>(g, x.total);
        if (x.total == 0) return out;
        const ExpandJob *dj = upload(g, x.jobs);
        const int nj = (int)x.jobs.size();
        const uint64_t total = x.total;
        dfacto_group *const grp = g;
        post.push_back([grp, dj, nj, total, out] {
            const unsigned grid = (unsigned)std::min<uint64_t>((total + 255) / 256, 8192);
            hipLaunchKernelGGL(k_expand<V>, dim3(grid), dim3(256), 0, grp->stream, dj, nj, total,
                               out);
            DF_LAUNCHED();
        });
        return out;
    }

    // One Gram over all members: out[t] = F(t)^T F(t) (rows(t) x R(t)).
    void add_gram(dfacto_dtype dt, const std::function<const void *(int)> &Fof,
                  const std::function<int64_t(int)> &rows_of,
                  const std::function<double *(int)> &out_of) {
        dfacto_group *const grp = g;  // lambdas outlive this builder: capture the group itself
        const int n = grp->n;
        std::vector<GramJob> jobs(n);
        std::map<std::pair<int, bool>, std::vector<uint2>> cls;  // (nt, vec) -> blocks
        std::vector<uint2> red;
        for (int t = 0; t < n; ++t) {
            const GramPlan p = gram_plan(rows_of(t), R[t], Fof(t), dt);
            jobs[t] = {Fof(t), rows_of(t), R[t], (uint32_t)p.nblk, ws[t].part, out_of(t)};
            auto &v = cls[{p.nt, p.vec}];
            for (int b = 0; b < p.nblk; ++b) v.push_back(make_uint2(t, b));
            for (uint32_t e = 0; e < gram_reduce_blocks(R[t]); ++e) red.push_back(make_uint2(t, e));
        }
        const GramJob *dj = upload(g, jobs);
        for (auto &kv : cls) {
            const uint2 *dvb = upload(g, kv.second);
            const int nt = kv.first.first;
            const bool vec = kv.first.second;
            const uint32_t nvb = (uint32_t)kv.second.size();
            grp->steps.push_back(
                [grp, dt, nt, vec, dj, dvb, nvb] { launch_gram_group(&grp->gctx, dt, nt, vec, dj, dvb, nvb); });
            ++g->launches;
        }
        const uint2 *dred = upload(g, red);
        const uint32_t nred = (uint32_t)red.size();
        grp->steps.push_back(
            [grp, dj, dred, nred] { launch_gram_reduce_group(&grp->gctx, dj, dred, nred); });
        ++g->launches;
    }

    void add_mode(int m) {
        dfacto_group *const grp = g;  // lambdas outlive this builder: capture the group itself
        const int n = grp->n;
        const dfacto_dtype dt = grp->dtype;
        // solve: H = G_p * G_q + reg I, Hinv
        {
            std::vector<SolveJob> jobs(n);
            const int p = (m + 1) % 3, q = (m + 2) % 3;
            for (int t = 0; t < n; ++t)
                jobs[t] = {R[t], reg, ws[t].G[p], ws[t].G[q], ws[t].Hinv, ws[t].solve_scratch,
                           ws[t].flag + m};
            const SolveJob *dj = upload(g, jobs);
            const int maxR = g->maxR;
            grp->steps.push_back(
                [grp, maxR, dj, n] { launch_solve_group(&grp->gctx, maxR, dj, (uint32_t)n); });
            ++g->launches;
        }
        // MTTKRP + fix-ups, one launch each per kernel class
        {
            std::vector<GroupMttkrp> desc(n);
            // relabeled members gather from copies of their factors in rank
            // order, permuted before the MTTKRP on the group's stream
            for (int t = 0; t < n; ++t) {
                if (!ws[t].perm) continue;
                const ModeData &md = T[t]->mode[m];
                const dfacto_tensor *tt = T[t];
                const int Rt = R[t];
                const void *Fl = F[3 * t + md.leaf], *Fm = F[3 * t + md.mid];
                void *buf = ws[t].perm;
                grp->steps.push_back([grp, tt, m, Rt, dt, Fl, Fm, buf] {
                    launch_relabeled_tables(&grp->gctx, tt, m, Rt, dt, Fl, Fm, buf);
                });
                g->launches += 2;
            }
            // launch forms per class: the default shape and, when tuning,
            // other columns per lane (fewer, or eight for BF16), lanes per
            // group to match, and 2 or 4 chunks per lane group; one
            // work-item table per item size
            const bool tune = tuning;
            auto forms = [tune, dt](const MttkrpShape &sh, const std::vector<int> &ranks) {
                std::vector<std::pair<MttkrpShape, unsigned>> f{{sh, 1u}};
                if (!tune) return f;
                std::vector<MttkrpShape> shapes{sh};
                // BF16 rows of a multiple of 8 columns: also 8 columns per
                // lane (one 16-byte load; the factors are 16-byte aligned)
                bool wide = dt == DFACTO_BF16 && sh.nch == 1 && sh.cpl < 8;
                for (int r : ranks) wide = wide && r % 8 == 0;
                const int top = wide ? 8 : sh.cpl / 2;
                for (int c = top; sh.nch == 1 && c >= 1; c /= 2) {
                    if (c == sh.cpl) continue;
                    // lanes per group: enough for the widest member (the
                    // lanes past a member's columns stay idle)
                    int lanes = 1;
                    for (int r : ranks) lanes = std::max(lanes, (r + c - 1) / c);
                    int gv = 2;
                    while (gv < lanes) gv <<= 1;
                    if (gv <= 64) shapes.push_back({c, gv, 1});
                }
                for (const MttkrpShape &x : shapes)
                    for (unsigned k : {1u, 2u, 4u})
                        if (!(x.cpl == sh.cpl && x.g == sh.g && k == 1)) f.push_back({x, k});
                return f;
            };
            struct Cls {
                MttkrpShape sh;
                bool small;
                std::vector<int> ranks;
                std::map<unsigned, Expansion<uint2>> items;  // by chunks per item
                Expansion<uint2> empty;
                Expansion<uint4> shortr, longr;
            };
            std::map<std::tuple<int, int, int, bool>, Cls> cls;
            for (int t = 0; t < n; ++t) {
                const ModeData &md = T[t]->mode[m];
                const void *Fl = F[3 * t + md.leaf], *Fm = F[3 * t + md.mid];
                if (ws[t].perm && md.perm_leaf)
                    relabeled_tables(T[t], m, R[t], dt, ws[t].perm, &Fl, &Fm);
                desc[t] = {md.stream, md.chunk_start, (uint32_t)md.nchunk, R[t], Fl, Fm,
                           ws[t].M, ws[t].carry};
                const MttkrpShape sh =
                    mttkrp_shape(R[t], dt, Fl, Fm, ws[t].M, ws[t].perm && md.perm_leaf);
                const bool sm = mttkrp_small(T[t], m);
                Cls &c = cls[{sh.cpl, sh.g, sh.nch, sm}];
                c.sh = sh;
                c.small = sm;
                c.ranks.push_back(R[t]);
                c.shortr.add(t, md.runs_short, md.nruns_short, 3, 0);
                c.longr.add(t, md.runs_long, md.nruns_long, 3, 0);
                c.empty.add(t, md.empty_rows, md.nempty, 1, 0);
            }
            // (t, first chunk) work items per item size, from each member's
            // chunk count; (t, row, first chunk, chunks) runs and (t, row)
            // empty rows from the members' own device lists
            for (auto &kv : cls) {
                Cls &c = kv.second;
                for (const auto &f : forms(c.sh, c.ranks)) {
                    const unsigned per = mttkrp_group_chunks_per_item(f.first, f.second);
                    if (c.items.count(per)) continue;
                    Expansion<uint2> &x = c.items[per];
                    for (int t = 0; t < n; ++t) {
                        const ModeData &md = T[t]->mode[m];
                        const MttkrpShape sh =
                            mttkrp_shape(R[t], dt, desc[t].Fleaf, desc[t].Fmid, ws[t].M,
                                         ws[t].perm && md.perm_leaf);
                        if (sh.cpl != c.sh.cpl || sh.g != c.sh.g || sh.nch != c.sh.nch ||
                            mttkrp_small(T[t], m) != c.small)
                            continue;
                        x.add(t, nullptr, (md.nchunk + per - 1) / per, 0, per);
                    }
                }
            }
            const GroupMttkrp *dd = upload(g, desc);
            for (auto &kv : cls) {
                Cls &c = kv.second;
                const MttkrpShape sh = c.sh;
                const bool sm = c.small;
                dfacto_group::MtLaunch L;
                L.small = sm;
                for (const auto &f : forms(c.sh, c.ranks)) {
                    const Expansion<uint2> &x = c.items[mttkrp_group_chunks_per_item(f.first, f.second)];
                    L.cands.push_back({f.first, f.second, nullptr, (uint32_t)x.total});
                }
                std::map<unsigned, const uint2 *> placed;
                for (auto &kv2 : c.items) placed[kv2.first] = expand(kv2.second);
                for (auto &v : L.cands) v.items = placed[mttkrp_group_chunks_per_item(v.sh, v.kper)];
                L.v = L.cands[0];
                L.grid = std::max(1u, std::min<unsigned>(L.v.nitems, (unsigned)g->gctx.num_cu * 8));
                g->mt.push_back(L);
                const size_t gi = g->mt.size() - 1;
                auto step = [grp, dt, dd, gi] {
                    const dfacto_group::MtLaunch &l = grp->mt[gi];
                    launch_mttkrp_group(&grp->gctx, dt, l.v.sh, l.small, dd, l.v.items,
                                        l.v.nitems, l.grid, l.v.kper);
                };
                g->steps.push_back(step);
                mt_steps.push_back(step);
                mt_index.push_back(gi);
                ++g->launches;
                const uint4 *ds = expand(c.shortr), *dl = expand(c.longr);
                const uint2 *de = expand(c.empty);
                const uint32_t ns = (uint32_t)c.shortr.total, ne = (uint32_t)c.empty.total,
                               nl = (uint32_t)c.longr.total;
                grp->steps.push_back([grp, sh, dd, ds, ns, de, ne, dl, nl] {
                    launch_fix_group(&grp->gctx, sh, dd, ds, ns, de, ne, dl, nl);
                });
                g->launches += (ns + ne > 0) + (nl > 0);
            }
        }
        // Gram of the MTTKRP result
        add_gram(
            DFACTO_F32, [&](int t) -> const void * { return ws[t].M; },
            [&](int t) { return T[t]->dims[m]; }, [&](int t) { return ws[t].MtM; });
        // lambda, new Gram, W, fit
        {
            std::vector<LambdaJob> jobs(n);
            for (int t = 0; t < n; ++t)
                jobs[t] = {R[t],       m,          ws[t].Hinv,     ws[t].MtM,      ws[t].G[m],
                           ws[t].W,    lambda[t],  ws[t].G[0],     ws[t].G[1],     T[t]->normsq,
                           fit + t,    ws[t].lam_scratch};
            const LambdaJob *dj = upload(g, jobs);
            const int maxR = g->maxR;
            grp->steps.push_back(
                [grp, maxR, dj, n] { launch_lambda_group(&grp->gctx, maxR, dj, (uint32_t)n); });
            ++g->launches;
        }
        // row map F_m = M W
        {
            std::vector<RowmapJob> jobs(n);
            std::map<std::pair<int, int>, std::vector<uint2>> cls;  // (kind, R) -> blocks
            for (int t = 0; t < n; ++t) {
                const RowmapPlan p = rowmap_plan(R[t], ws[t].M, F[3 * t + m], dt, T[t]->dims[m]);
                if (p.kind == RowmapPlan::kGeneric)
                    throw Error{DFACTO_E_UNSUPPORTED, "no grouped row map for this rank"};
                jobs[t] = {ws[t].M, T[t]->dims[m], ws[t].W, F[3 * t + m], p.nblk};
                auto &v = cls[{p.kind, R[t]}];
                for (uint32_t b = 0; b < p.nblk; ++b) v.push_back(make_uint2(t, b));
            }
            const RowmapJob *dj = upload(g, jobs);
            for (auto &kv : cls) {
                const uint2 *dvb = upload(g, kv.second);
                const int kind = kv.first.first, Rc = kv.first.second;
                const uint32_t nvb = (uint32_t)kv.second.size();
                grp->steps.push_back([grp, dt, kind, Rc, dj, dvb, nvb] {
                    launch_rowmap_group(&grp->gctx, dt, kind, Rc, dj, dvb, nvb);
                });
                ++g->launches;
            }
        }
        // BF16 storage: later modes use the Gram of the stored factor, and
        // the fit is that of the stored factors
        if (dt == DFACTO_BF16) {
            add_gram(
                DFACTO_BF16, [&](int t) -> const void * { return F[3 * t + m]; },
                [&](int t) { return T[t]->dims[m]; }, [&](int t) { return ws[t].G[m]; });
            if (m == 2) add_fit();
        }
    }

    // fit of the stored factors, every member: (member, block) partial sums
    // of <C diag(lambda), M> into the member's Gram partial buffer (free
    // again once the Gram above is reduced), then one block per member
    void add_fit() {
        dfacto_group *const grp = g;
        const int n = grp->n;
        std::vector<FitJob> jobs(n);
        std::vector<uint2> items;
        for (int t = 0; t < n; ++t) {
            const int64_t rows = T[t]->dims[2];
            const uint32_t nb = fit_blocks(rows, R[t]);
            jobs[t] = {F[3 * t + 2], ws[t].M, rows, R[t], nb, lambda[t], ws[t].G[0],
                       ws[t].G[1], ws[t].G[2], T[t]->normsq, ws[t].part, fit + t};
            for (uint32_t b = 0; b < nb; ++b) items.push_back(make_uint2(t, b));
        }
        const FitJob *dj = upload(g, jobs);
        const uint2 *di = upload(g, items);
        const uint32_t ni = (uint32_t)items.size();
        const dfacto_dtype dt = grp->dtype;
        grp->steps.push_back(
            [grp, dt, dj, n, di, ni] { launch_fit_group(&grp->gctx, dt, dj, (uint32_t)n, di, ni); });
        g->launches += 2;
    }
};

void run_steps(dfacto_group *g, size_t from) {
    for (size_t k = from; k < g->steps.size(); ++k) g->steps[k]();
}

void drop_graphs(dfacto_group *g) {
    for (int q = 0; q < 2; ++q) {
        if (g->exec[q]) (void)hipGraphExecDestroy(g->exec[q]);
        if (g->graph[q]) (void)hipGraphDestroy(g->graph[q]);
        g->exec[q] = nullptr;
        g->graph[q] = nullptr;
    }
}

// Time the MTTKRP steps of the group and keep the fastest launch form per
// kernel class: first the persistent grid size of the default form (2 to 32
// workgroups per CU), then every other form (shape, chunks per lane group)
// at that grid, then the grid again for the winner.  Only the MTTKRP kernels
// run (they write the group's own workspace, never the factors).
void autotune(dfacto_group *g, const std::vector<std::function<void()>> &mt_steps,
              const std::vector<size_t> &mt_index) {
    hipEvent_t e0, e1;
    DF_HIP(hipEventCreate(&e0));
    DF_HIP(hipEventCreate(&e1));
    const unsigned cu = (unsigned)std::max(1, g->gctx.num_cu);
    for (size_t k = 0; k < mt_steps.size(); ++k) {
        dfacto_group::MtLaunch &L = g->mt[mt_index[k]];
        mt_steps[k]();  // warm the class's data once
        auto time_it = [&]() {
            DF_HIP(hipEventRecord(e0, g->stream));
            mt_steps[k]();
            DF_HIP(hipEventRecord(e1, g->stream));
            DF_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            DF_HIP(hipEventElapsedTime(&ms, e0, e1));
            return ms;
        };
        auto clamp = [&](unsigned want) {
            return std::max(1u, std::min<unsigned>(want, std::max<uint32_t>(L.v.nitems, 1u)));
        };
        float best_ms = 1e30f;
        dfacto_group::MtVariant best_v = L.v;
        unsigned best_grid = L.grid;
        auto grid_sweep = [&]() {
            for (unsigned per_cu : {2u, 4u, 8u, 16u, 32u}) {
                L.grid = clamp(cu * per_cu);
                const float ms = time_it();
                if (ms < best_ms) best_ms = ms, best_v = L.v, best_grid = L.grid;
            }
        };
        grid_sweep();
        const unsigned grid0 = best_grid;
        for (size_t c = 1; c < L.cands.size(); ++c) {
            L.v = L.cands[c];
            L.grid = clamp(grid0);
            const float ms = time_it();
            if (ms < best_ms) best_ms = ms, best_v = L.v, best_grid = L.grid;
        }
        if (best_v.sh.cpl != L.cands[0].sh.cpl || best_v.sh.g != L.cands[0].sh.g ||
            best_v.kper != L.cands[0].kper) {
            L.v = best_v;
            grid_sweep();
        }
        L.v = best_v;
        L.grid = best_grid;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

}  // namespace

using namespace dfacto;

extern "C" {

dfacto_status dfacto_group_create(dfacto_ctx *ctx, int n, const dfacto_tensor *const *tensors,
                                  const int *ranks, dfacto_dtype dtype, double reg,
                                  void *const *d_F, double *const *d_lambda, double *d_fit,
                                  int flags, dfacto_group **out) {
    return guarded(ctx, [&] {
        if (!out) throw Error{DFACTO_E_INVALID, "out is NULL"};
        *out = nullptr;
        if (n < 1) throw Error{DFACTO_E_INVALID, "a group needs at least one member"};
        if (!tensors || !ranks || !d_F || !d_lambda || !d_fit)
            throw Error{DFACTO_E_INVALID, "NULL argument"};
        if (!(reg >= 0.0)) throw Error{DFACTO_E_INVALID, "reg must be >= 0"};
        if ((flags & DFACTO_GROUP_CTX_STREAM) && (flags & DFACTO_GROUP_GRAPH) && !ctx->stream)
            throw Error{DFACTO_E_INVALID, "graph capture needs a created stream, not the null stream"};
        hip_check(hipGetLastError(), "a HIP call before dfacto_group_create");
        std::vector<const dfacto_tensor *> T(tensors, tensors + n);
        std::vector<int> R(ranks, ranks + n);
        for (int t = 0; t < n; ++t) {
            check_common(T[t], R[t], dtype);
            if (T[t]->device != ctx->device)
                throw Error{DFACTO_E_INVALID, "group member built on another device"};
            if (!group_rank_ok(R[t]))
                throw Error{DFACTO_E_UNSUPPORTED,
                            "grouped ALS supports R in {4, 8, 12, 16, 32, 48, 64}"};
            for (int m = 0; m < 3; ++m) {
                if (!d_F[3 * t + m]) throw Error{DFACTO_E_INVALID, "factor is NULL"};
                if ((uintptr_t)d_F[3 * t + m] % 16)
                    throw Error{DFACTO_E_INVALID, "grouped factors must be 16-byte aligned"};
            }
            if (!d_lambda[t]) throw Error{DFACTO_E_INVALID, "lambda is NULL"};
        }
        dfacto_group *g = new dfacto_group();
        try {
            g->device = ctx->device;
            g->n = n;
            g->dtype = dtype;
            g->maxR = *std::max_element(R.begin(), R.end());
            g->use_graph = (flags & DFACTO_GROUP_GRAPH) != 0;
            g->own_stream = (flags & DFACTO_GROUP_CTX_STREAM) == 0;
            g->mem = ctx->mem;
            if (g->own_stream) DF_HIP(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking));
            else g->stream = ctx->stream;
            g->gctx.device = ctx->device;
            g->gctx.num_cu = ctx->num_cu;
            g->gctx.stream = g->stream;
            if (g->own_stream) {  // inputs (tensors, factors) come from ctx's stream
                DF_HIP(hipEventCreateWithFlags(&g->ev_in, hipEventDisableTiming));
                DF_HIP(hipEventCreateWithFlags(&g->ev_out, hipEventDisableTiming));
                DF_HIP(hipEventRecord(g->ev_in, ctx->stream));
                DF_HIP(hipStreamWaitEvent(g->stream, g->ev_in, 0));
            }

            Build b{g, T, R, reg, d_F, d_lambda, d_fit, {}};
            b.tuning = (flags & DFACTO_GROUP_TUNE) != 0;
            b.ws.resize(n);
            // one allocation for every member's workspace: per member the
            // MTTKRP output (largest mode), the carries (most chunks) and the
            // FP64 R x R block, each starting on a 256-byte boundary
            auto al = [](size_t bytes) { return (bytes + 255) & ~(size_t)255; };
            std::vector<size_t> off_M(n), off_carry(n), off_d(n), off_p(n);
            size_t total = 0;
            for (int t = 0; t < n; ++t) {
                const size_t RR = (size_t)R[t] * R[t];
                int64_t dmax = 0, cmax = 1;
                for (int m = 0; m < 3; ++m) {
                    dmax = std::max(dmax, T[t]->dims[m]);
                    cmax = std::max(cmax, T[t]->mode[m].nchunk);
                }
                off_M[t] = total, total += al(4 * (size_t)dmax * R[t]);
                off_carry[t] = total, total += al(4 * (size_t)cmax * R[t]);
                off_d[t] = total, total += al(8 * (6 * RR + 3 * RR + (4 * RR + R[t]) + 256 * RR + 8));
                const size_t pb = perm_bytes(T[t], R[t], dtype);
                off_p[t] = pb ? total : 0;
                total += al(pb);
            }
            char *base = dev_alloc<char>(g, total);
            for (int t = 0; t < n; ++t) {
                const size_t RR = (size_t)R[t] * R[t];
                MemberWs &w = b.ws[t];
                w.M = (float *)(base + off_M[t]);
                w.carry = (float *)(base + off_carry[t]);
                w.perm = off_p[t] ? base + off_p[t] : nullptr;
                double *d = (double *)(base + off_d[t]);
                size_t o = 0;
                for (int m = 0; m < 3; ++m) w.G[m] = d + o, o += RR;
                w.Hinv = d + o, o += RR;
                w.W = d + o, o += RR;
                w.MtM = d + o, o += RR;
                w.solve_scratch = d + o, o += 3 * RR;
                w.lam_scratch = d + o, o += 4 * RR + R[t];
                w.part = d + o, o += 256 * RR;
                w.flag = (int *)(d + o);
            }
            // iteration: Grams of B and C, then modes 0, 1, 2
            for (int m = 1; m < 3; ++m)
                b.add_gram(
                    dtype, [&](int t) -> const void * { return d_F[3 * t + m]; },
                    [&](int t) { return T[t]->dims[m]; }, [&](int t) { return b.ws[t].G[m]; });
            g->open_end = g->steps.size();
            g->reuse_grams = dtype == DFACTO_BF16;
            g->own_factors = (flags & DFACTO_GROUP_OWN_FACTORS) != 0;
            for (int m = 0; m < 3; ++m) b.add_mode(m);
            // the host tables in one copy per arena chunk, then the combined
            // tables expanded on the device (stream order keeps them ahead of
            // every iteration)
            upload_all(g);
            for (auto &f : b.post) f();

            if (flags & DFACTO_GROUP_TUNE) autotune(g, b.mt_steps, b.mt_index);
            *out = g;
        } catch (...) {
            dfacto_group_destroy(g);
            throw;
        }
    });
}

dfacto_status dfacto_group_als(dfacto_ctx *ctx, dfacto_group *g, int iters) {
    return guarded(ctx, [&] {
        if (!g) throw Error{DFACTO_E_INVALID, "group is NULL"};
        if (g->device != ctx->device) throw Error{DFACTO_E_INVALID, "group on another device"};
        if (!g->own_stream && g->stream != ctx->stream)
            throw Error{DFACTO_E_INVALID, "group launches on its creating context's stream"};
        if (iters < 0) throw Error{DFACTO_E_INVALID, "iters must be >= 0"};
        hip_check(hipGetLastError(), "a HIP call before dfacto_group_als");
        if (g->own_stream) {
            DF_HIP(hipEventRecord(g->ev_in, ctx->stream));
            DF_HIP(hipStreamWaitEvent(g->stream, g->ev_in, 0));
        }
        for (int i = 0; i < iters; ++i) {
            const int q = g->reuse_grams && (i > 0 || (g->own_factors && g->grams_valid)) ? 1 : 0;
            const size_t from = q ? g->open_end : 0;
            if (!g->use_graph) {
                run_steps(g, from);
                continue;
            }
            if (!g->exec[q]) {
                DF_HIP(hipStreamBeginCapture(g->stream, hipStreamCaptureModeRelaxed));
                try {
                    run_steps(g, from);
                } catch (...) {
                    hipGraph_t tmp = nullptr;
                    (void)hipStreamEndCapture(g->stream, &tmp);
                    if (tmp) (void)hipGraphDestroy(tmp);
                    throw;
                }
                DF_HIP(hipStreamEndCapture(g->stream, &g->graph[q]));
                DF_HIP(hipGraphInstantiate(&g->exec[q], g->graph[q], nullptr, nullptr, 0));
            }
            DF_HIP(hipGraphLaunch(g->exec[q], g->stream));
        }
        if (iters > 0) g->grams_valid = true;
        if (g->own_stream) {
            DF_HIP(hipEventRecord(g->ev_out, g->stream));
            DF_HIP(hipStreamWaitEvent(ctx->stream, g->ev_out, 0));
        }
    });
}

dfacto_status dfacto_group_get_info(const dfacto_group *g, dfacto_group_info *info) {
    if (!g || !info) return DFACTO_E_INVALID;
    info->members = g->n;
    info->launches_per_iter = g->launches;
    info->bytes = g->bytes;
    info->graph = g->use_graph ? 1 : 0;
    info->mttkrp_classes = (int)g->mt.size();
    for (int k = 0; k < 16; ++k) {
        const bool have = k < (int)g->mt.size();
        info->mttkrp_grid[k] = have ? (int)g->mt[k].grid : 0;
        info->mttkrp_cpl[k] = have ? g->mt[k].v.sh.cpl : 0;
        info->mttkrp_lanes[k] = have ? g->mt[k].v.sh.g : 0;
        info->mttkrp_chunks_per_group[k] = have ? (int)g->mt[k].v.kper : 0;
        info->mttkrp_forms[k] = have ? (int)g->mt[k].cands.size() : 0;
    }
    return DFACTO_OK;
}

dfacto_status dfacto_group_set_form(dfacto_group *g, int cls, int form, int grid) {
    if (!g || cls < 0 || cls >= (int)g->mt.size()) return DFACTO_E_INVALID;
    dfacto_group::MtLaunch &L = g->mt[cls];
    if (form < 0 || form >= (int)L.cands.size() || grid < 1) return DFACTO_E_INVALID;
    L.v = L.cands[form];
    L.grid = (unsigned)grid;
    drop_graphs(g);  // the captured iterations hold the old launch: capture again
    return DFACTO_OK;
}

void dfacto_group_destroy(dfacto_group *g) {
    if (!g) return;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(g->device);
    drop_graphs(g);
    for (void *p : g->allocs) g->mem.free(p, g->stream);
    if (g->stream || !g->own_stream) (void)hipStreamSynchronize(g->stream);  // host tables
    if (g->ev_in) (void)hipEventDestroy(g->ev_in);
    if (g->ev_out) (void)hipEventDestroy(g->ev_out);
    if (g->stream && g->own_stream) (void)hipStreamDestroy(g->stream);
    if (prev >= 0) (void)hipSetDevice(prev);
    delete g;
}

}  // extern "C"
