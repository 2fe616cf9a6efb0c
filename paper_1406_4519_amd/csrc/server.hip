// server.hip -- served CP-ALS solves with continuous batching.
//
// A server owns one worker thread, a HIP stream and a device-memory budget.
// Clients submit solve requests (host COO, rank, storage dtype, initial
// factors, stopping rule) at any time.  At every iteration boundary the
// worker
//   1. admits queued requests in arrival order while their device footprint
//      fits the budget and a slot is free: it uploads the COO, builds the
//      flattenings and uploads the initial factors;
//   2. runs one CP-ALS iteration (Algorithm 2) of every active request as a
//      group (grouped launches, one group per storage dtype and ridge value);
//   3. reads the fits and retires every request whose fit changed by less
//      than its tolerance or that reached its iteration cap: factors and
//      lambda are copied to the caller's host buffers and its memory is
//      freed, which lets the next queued requests in.
// Requests that arrive while others run join at the next boundary, so work
// of different requests overlaps on the device.  A member's arithmetic does
// not depend on the other members (grouped launches reproduce the
// single-tensor results bit for bit), so every result is the same alone and
// in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.hpp"

namespace {
using namespace dfacto;
using Clock = std::chrono::steady_clock;

uint16_t host_f32_to_bf16(float f) {  // nearest, ties to even (NaN kept quiet)
    uint32_t b;
    std::memcpy(&b, &f, 4);
    if ((b & 0x7F800000u) == 0x7F800000u) return (uint16_t)((b >> 16) | ((b & 0xFFFFu) ? 0x40u : 0u));
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

float host_bf16_to_f32(uint16_t h) {
    const uint32_t b = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &b, 4);
    return f;
}

struct Member {
    int64_t id = 0;
    dfacto_request req{};
    dfacto_request_status st{};
    Clock::time_point t_submit;
    dfacto_tensor *tensor = nullptr;
    void *F[3] = {nullptr, nullptr, nullptr};
    double *lambda = nullptr;
    size_t footprint = 0;  // device bytes held while active
    double prev_fit = 0.0;
    bool has_prev = false;
};

}  // namespace

struct dfacto_server {
    int device = 0;
    size_t budget = 0;
    int max_slots = 1;
    dfacto_ctx *ctx = nullptr;  // the worker's context (own stream)
    hipStream_t stream = nullptr;
    Clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    int64_t next_id = 1;
    std::deque<std::unique_ptr<Member>> pending;
    std::map<int64_t, dfacto_request_status> finished;  // id -> final status
    std::map<int64_t, int> running;                     // ids admitted and not yet done

    // worker-only state
    std::vector<std::unique_ptr<Member>> active;
    std::vector<dfacto_group *> groups;  // over `active`, rebuilt when it changes
    bool dirty = true;
    size_t used = 0;
    int peak_active = 0;
    int64_t iterations = 0;
    double *d_fits = nullptr;  // max_slots doubles
    std::thread worker;
};

namespace {

double seconds_since(const dfacto_server *s, Clock::time_point t) {
    return std::chrono::duration<double>(t - s->t0).count();
}

// Device bytes a request holds while active: its flattenings (at most two
// 8-byte entries per nonzero per mode, plus chunk and run tables), its
// factors, lambda and the group's per-member workspace (MTTKRP output and
// carries, R x R matrices and Gram partial sums).
size_t footprint_estimate(const dfacto_request &r) {
    const size_t es = r.dtype == DFACTO_BF16 ? 2 : 4;
    const size_t R = (size_t)r.R;
    const size_t nnz = (size_t)r.nnz;
    int64_t dmax = std::max(r.dims[0], std::max(r.dims[1], r.dims[2]));
    size_t b = 3 * (16 * nnz + 16 * (nnz / 256 + 2) + 4 * (size_t)dmax) + 3 * 64 * 8;
    for (int m = 0; m < 3; ++m) b += (size_t)r.dims[m] * R * es;
    b += R * 8;
    b += (size_t)dmax * R * 4 + (nnz / 256 + 2) * R * 4 + (256 + 16) * R * R * 8;
    return b;
}

// Peak transient device memory of building the flattenings (COO staging,
// sort keys and permutations, gathered copies).
size_t build_transient(const dfacto_request &r) { return 80 * (size_t)r.nnz + (1 << 20); }

void free_member(Member &m) {
    for (int k = 0; k < 3; ++k)
        if (m.F[k]) (void)hipFree(m.F[k]), m.F[k] = nullptr;
    if (m.lambda) (void)hipFree(m.lambda), m.lambda = nullptr;
    if (m.tensor) dfacto_tensor_destroy(m.tensor), m.tensor = nullptr;
}

void finish(dfacto_server *s, std::unique_ptr<Member> mp, dfacto_status status) {
    Member &m = *mp;
    m.st.status = status;
    m.st.done = 1;
    m.st.t_done = seconds_since(s, Clock::now());
    std::lock_guard<std::mutex> lk(s->mu);
    s->running.erase(m.id);
    s->finished[m.id] = m.st;
    s->cv_done.notify_all();
}

// Upload, build and initialize one request on the worker's stream.
void admit(dfacto_server *s, Member &m) {
    const dfacto_request &r = m.req;
    hipStream_t st = s->stream;
    uint32_t *di = nullptr, *dj = nullptr, *dk = nullptr;
    float *dv = nullptr;
    const size_t n = (size_t)std::max<int64_t>(r.nnz, 1);
    auto cleanup = [&] {
        (void)hipFree(di), (void)hipFree(dj), (void)hipFree(dk), (void)hipFree(dv);
    };
    try {
        hip_check(hipMalloc(&di, 4 * n), "request upload");
        hip_check(hipMalloc(&dj, 4 * n), "request upload");
        hip_check(hipMalloc(&dk, 4 * n), "request upload");
        hip_check(hipMalloc(&dv, 4 * n), "request upload");
        if (r.nnz > 0) {
            DF_HIP(hipMemcpyAsync(di, r.i, 4 * r.nnz, hipMemcpyHostToDevice, st));
            DF_HIP(hipMemcpyAsync(dj, r.j, 4 * r.nnz, hipMemcpyHostToDevice, st));
            DF_HIP(hipMemcpyAsync(dk, r.k, 4 * r.nnz, hipMemcpyHostToDevice, st));
            DF_HIP(hipMemcpyAsync(dv, r.val, 4 * r.nnz, hipMemcpyHostToDevice, st));
        }
        const dfacto_status bs =
            dfacto_build_flattenings(s->ctx, r.dims, r.nnz, di, dj, dk, dv, &m.tensor);
        if (bs != DFACTO_OK) throw Error{bs, dfacto_last_error(s->ctx)};
        cleanup();
        di = dj = dk = nullptr;
        dv = nullptr;
        const size_t es = r.dtype == DFACTO_BF16 ? 2 : 4;
        for (int k = 0; k < 3; ++k) {
            const size_t cnt = (size_t)r.dims[k] * r.R;
            hip_check(hipMalloc(&m.F[k], std::max<size_t>(es * cnt, 16)), "factor allocation");
            if (r.dtype == DFACTO_BF16) {
                std::vector<uint16_t> h(cnt);
                for (size_t e = 0; e < cnt; ++e) h[e] = host_f32_to_bf16(r.init[k][e]);
                DF_HIP(hipMemcpy(m.F[k], h.data(), 2 * cnt, hipMemcpyHostToDevice));
            } else {
                DF_HIP(hipMemcpy(m.F[k], r.init[k], 4 * cnt, hipMemcpyHostToDevice));
            }
        }
        hip_check(hipMalloc(&m.lambda, 8 * (size_t)r.R), "lambda allocation");
        m.footprint = std::max(m.footprint, m.tensor->bytes + footprint_estimate(r) -
                                                3 * 16 * (size_t)r.nnz);
    } catch (...) {
        cleanup();
        throw;
    }
}

// Copy a finished request's factors and lambda to its host buffers.
void deliver(dfacto_server *s, Member &m) {
    const dfacto_request &r = m.req;
    for (int k = 0; k < 3; ++k) {
        const size_t cnt = (size_t)r.dims[k] * r.R;
        if (!r.out_F[k]) continue;
        if (r.dtype == DFACTO_BF16) {
            std::vector<uint16_t> h(cnt);
            DF_HIP(hipMemcpy(h.data(), m.F[k], 2 * cnt, hipMemcpyDeviceToHost));
            for (size_t e = 0; e < cnt; ++e) r.out_F[k][e] = host_bf16_to_f32(h[e]);
        } else {
            DF_HIP(hipMemcpy(r.out_F[k], m.F[k], 4 * cnt, hipMemcpyDeviceToHost));
        }
    }
    if (r.out_lambda) DF_HIP(hipMemcpy(r.out_lambda, m.lambda, 8 * (size_t)r.R, hipMemcpyDeviceToHost));
    (void)s;
}

void drop_groups(dfacto_server *s) {
    for (dfacto_group *g : s->groups) dfacto_group_destroy(g);
    s->groups.clear();
    s->dirty = true;
}

// One CP-ALS iteration of every active request.  The active list is kept
// ordered by (dtype, reg); each run of one class is one group, and a
// class's members own consecutive fit slots.  The groups are rebuilt only
// when the active set changes.
void iterate(dfacto_server *s) {
    if (s->dirty) {
        drop_groups(s);
        std::stable_sort(s->active.begin(), s->active.end(),
                         [](const std::unique_ptr<Member> &a, const std::unique_ptr<Member> &b) {
                             if (a->req.dtype != b->req.dtype) return a->req.dtype < b->req.dtype;
                             return a->req.reg < b->req.reg;
                         });
        size_t a = 0;
        while (a < s->active.size()) {
            size_t b = a;
            const dfacto_dtype dt = s->active[a]->req.dtype;
            const double reg = s->active[a]->req.reg;
            std::vector<const dfacto_tensor *> T;
            std::vector<int> R;
            std::vector<void *> F;
            std::vector<double *> lam;
            while (b < s->active.size() && s->active[b]->req.dtype == dt &&
                   s->active[b]->req.reg == reg) {
                Member &m = *s->active[b];
                T.push_back(m.tensor);
                R.push_back(m.req.R);
                for (int k = 0; k < 3; ++k) F.push_back(m.F[k]);
                lam.push_back(m.lambda);
                ++b;
            }
            dfacto_group *g = nullptr;
            const dfacto_status st =
                dfacto_group_create(s->ctx, (int)T.size(), T.data(), R.data(), dt, reg, F.data(),
                                    lam.data(), s->d_fits + a, 0, &g);
            if (st != DFACTO_OK) throw Error{st, dfacto_last_error(s->ctx)};
            s->groups.push_back(g);
            a = b;
        }
        s->dirty = false;
    }
    for (dfacto_group *g : s->groups) {
        const dfacto_status st = dfacto_group_als(s->ctx, g, 1);
        if (st != DFACTO_OK) throw Error{st, dfacto_last_error(s->ctx)};
    }
}

void worker_main(dfacto_server *s) {
    (void)hipSetDevice(s->device);
    for (;;) {
        // admission
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stop || !s->pending.empty() || !s->active.empty(); });
            if (s->stop && s->pending.empty() && s->active.empty()) return;
        }
        for (;;) {
            std::unique_ptr<Member> m;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                if (s->pending.empty() || (int)s->active.size() >= s->max_slots) break;
                Member &f = *s->pending.front();
                const size_t need = footprint_estimate(f.req) + build_transient(f.req);
                // the first request is admitted even when it alone exceeds
                // the budget (it fails with E_NOMEM if the device cannot hold it)
                if (!s->active.empty() && s->used + need > s->budget) break;
                m = std::move(s->pending.front());
                s->pending.pop_front();
                s->running[m->id] = 1;
            }
            m->st.t_admit = seconds_since(s, Clock::now());
            m->footprint = footprint_estimate(m->req);
            try {
                admit(s, *m);
            } catch (const Error &e) {
                free_member(*m);
                finish(s, std::move(m), e.code);
                continue;
            }
            s->used += m->footprint;
            drop_groups(s);  // the groups refer to the old active set
            s->active.push_back(std::move(m));
            s->peak_active = std::max(s->peak_active, (int)s->active.size());
        }
        if (s->active.empty()) continue;
        // one iteration for everyone, then the stopping rule per request
        try {
            iterate(s);
            std::vector<double> fits(s->active.size());
            DF_HIP(hipMemcpyAsync(fits.data(), s->d_fits, 8 * fits.size(), hipMemcpyDeviceToHost,
                                  s->stream));
            DF_HIP(hipStreamSynchronize(s->stream));
            ++s->iterations;
            std::vector<std::unique_ptr<Member>> keep;
            for (size_t a = 0; a < s->active.size(); ++a) {
                std::unique_ptr<Member> &m = s->active[a];
                m->st.iters += 1;
                m->st.fit = fits[a];
                const bool conv = m->has_prev && std::fabs(fits[a] - m->prev_fit) < m->req.tol;
                m->prev_fit = fits[a];
                m->has_prev = true;
                if (conv || m->st.iters >= m->req.max_iters) {
                    if (!s->groups.empty()) drop_groups(s);
                    dfacto_status code = DFACTO_OK;
                    try {
                        deliver(s, *m);
                    } catch (const Error &e) {
                        code = e.code;
                    }
                    s->used -= std::min(s->used, m->footprint);
                    free_member(*m);
                    finish(s, std::move(m), code);
                } else {
                    keep.push_back(std::move(m));
                }
            }
            s->active.swap(keep);
        } catch (const Error &e) {
            // a device failure ends every active request with its code
            drop_groups(s);
            for (auto &m : s->active) {
                free_member(*m);
                finish(s, std::move(m), e.code);
            }
            s->active.clear();
            s->used = 0;
        }
    }
}

}  // namespace

using namespace dfacto;

extern "C" {

dfacto_status dfacto_server_create(int device, size_t hbm_budget, int max_slots,
                                   dfacto_server **out) {
    if (!out || max_slots < 1) return DFACTO_E_INVALID;
    *out = nullptr;
    dfacto_server *s = new (std::nothrow) dfacto_server();
    if (!s) return DFACTO_E_NOMEM;
    s->device = device;
    s->max_slots = max_slots;
    s->t0 = Clock::now();
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(device) != hipSuccess ||
        hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return DFACTO_E_DEVICE;
    }
    if (hbm_budget == 0) {  // default: 90% of the free device memory
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess) hbm_budget = fr / 10 * 9;
    }
    s->budget = hbm_budget;
    if (hipMalloc(&s->d_fits, 8 * (size_t)max_slots) != hipSuccess ||
        dfacto_ctx_create(device, s->stream, &s->ctx) != DFACTO_OK) {
        (void)hipGetLastError();
        if (s->d_fits) (void)hipFree(s->d_fits);
        (void)hipStreamDestroy(s->stream);
        delete s;
        return DFACTO_E_DEVICE;
    }
    if (prev >= 0) (void)hipSetDevice(prev);
    s->worker = std::thread(worker_main, s);
    *out = s;
    return DFACTO_OK;
}

dfacto_status dfacto_server_submit(dfacto_server *s, const dfacto_request *req, int64_t *id) {
    if (!s || !req || !id) return DFACTO_E_INVALID;
    const dfacto_request &r = *req;
    if (r.nnz < 0 || r.dims[0] < 1 || r.dims[1] < 1 || r.dims[2] < 1) return DFACTO_E_INVALID;
    if (r.nnz > 0 && (!r.i || !r.j || !r.k || !r.val)) return DFACTO_E_INVALID;
    if (!r.init[0] || !r.init[1] || !r.init[2]) return DFACTO_E_INVALID;
    if (r.dtype != DFACTO_F32 && r.dtype != DFACTO_BF16) return DFACTO_E_INVALID;
    if (!(r.reg >= 0.0) || !(r.tol >= 0.0) || r.max_iters < 1) return DFACTO_E_INVALID;
    if (!(r.R == 4 || r.R == 8 || r.R == 12 || r.R == 16 || r.R == 32 || r.R == 48 || r.R == 64))
        return DFACTO_E_UNSUPPORTED;
    auto m = std::make_unique<Member>();
    m->req = r;
    m->t_submit = Clock::now();
    m->st.t_submit = seconds_since(s, m->t_submit);
    std::lock_guard<std::mutex> lk(s->mu);
    m->id = s->next_id++;
    *id = m->id;
    s->pending.push_back(std::move(m));
    s->cv_work.notify_one();
    return DFACTO_OK;
}

dfacto_status dfacto_server_poll(dfacto_server *s, int64_t id, dfacto_request_status *st) {
    if (!s || !st) return DFACTO_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->finished.find(id);
    if (it != s->finished.end()) {
        *st = it->second;
        return DFACTO_OK;
    }
    if (id < 1 || id >= s->next_id) return DFACTO_E_INVALID;
    return DFACTO_E_AGAIN;
}

dfacto_status dfacto_server_wait(dfacto_server *s, int64_t id, dfacto_request_status *st) {
    if (!s || !st) return DFACTO_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    if (id < 1 || id >= s->next_id) return DFACTO_E_INVALID;
    s->cv_done.wait(lk, [&] { return s->finished.count(id) > 0; });
    *st = s->finished[id];
    return DFACTO_OK;
}

dfacto_status dfacto_server_get_stats(dfacto_server *s, dfacto_server_stats *out) {
    if (!s || !out) return DFACTO_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    out->pending = (int64_t)s->pending.size();
    out->running = (int64_t)s->running.size();
    out->finished = (int64_t)s->finished.size();
    out->peak_active = s->peak_active;
    out->iterations = s->iterations;
    out->budget = s->budget;
    return DFACTO_OK;
}

void dfacto_server_destroy(dfacto_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    drop_groups(s);
    for (auto &m : s->active) free_member(*m);
    if (s->ctx) dfacto_ctx_destroy(s->ctx);
    if (s->d_fits) (void)hipFree(s->d_fits);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    if (prev >= 0) (void)hipSetDevice(prev);
    delete s;
}

}  // extern "C"
