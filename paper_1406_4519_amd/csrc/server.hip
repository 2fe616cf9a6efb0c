// server.hip -- served CP-ALS solves with continuous batching.
//
// A server owns a worker thread and kBuilders builder threads, each with
// its own HIP stream, and a device-memory budget.  Clients submit solve
// requests (host COO, rank, storage dtype, initial factors, stopping rule)
// at any time.
//   - A builder admits queued requests in arrival order while a slot is
//     free and their device footprint fits the budget (slots and bytes are
//     reserved at admission): it uploads the COO, builds the flattenings and
//     uploads the initial factors on its own stream, then hands the request
//     to the worker.  Building overlaps with the running iterations and with
//     the other builder's host-side work.
//   - At every iteration boundary the worker attaches the built requests,
//     runs one CP-ALS iteration (Algorithm 2) of every active request as a
//     group (grouped launches, one group per storage dtype and ridge value),
//     reads the fits and retires every request whose fit changed by less
//     than its tolerance or that reached its iteration cap.
//   - A delivery thread copies a retired request's factors and lambda to the
//     caller's host buffers and releases its memory (stream-ordered, without
//     waiting for the other requests' work), which frees its slot and bytes
//     for the next queued requests.
// Requests that arrive while others run join at the next boundary after
// their build, so work of different requests overlaps on the device.  A member's arithmetic does
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

// FP32 -> BF16, nearest with ties to even (a NaN stays a quiet NaN)
__global__ void k_f32_to_bf16(const float *__restrict__ in, uint16_t *__restrict__ out,
                              int64_t n) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        uint32_t b = __float_as_uint(in[e]);
        if ((b & 0x7F800000u) == 0x7F800000u) {
            out[e] = (uint16_t)((b >> 16) | ((b & 0xFFFFu) ? 0x40u : 0u));
        } else {
            b += 0x7FFFu + ((b >> 16) & 1u);
            out[e] = (uint16_t)(b >> 16);
        }
    }
}

__global__ void k_bf16_to_f32(const uint16_t *__restrict__ in, float *__restrict__ out,
                              int64_t n) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        out[e] = __uint_as_float((uint32_t)in[e] << 16);
}

unsigned convert_grid(int64_t n) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192));
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
    hipStream_t mem_stream = nullptr;  // stream the member's memory is ordered on
};

// Host-device copies through two pinned host buffers in turn.  Copies from
// the caller's pageable memory otherwise go through the runtime's own small
// staging copies (tens per request); here the host copies a chunk of up to
// kBytes into a pinned buffer while the device copies the previous one.
// BF16 factors are converted chunk by chunk in a device buffer of the ring,
// so a request makes no allocation for the conversion.  One ring per thread
// that copies (each builder, the delivery thread).
struct Staging {
    static constexpr size_t kBytes = (size_t)32 << 20;
    void *buf[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    float *dev = nullptr;  // kBytes on the device: one FP32 chunk being converted
    int next = 0;
    bool init() {
        for (int k = 0; k < 2; ++k)
            if (hipHostMalloc(&buf[k], kBytes, hipHostMallocDefault) != hipSuccess ||
                hipEventCreateWithFlags(&ev[k], hipEventDisableTiming) != hipSuccess) {
                (void)hipGetLastError();
                return false;
            }
        if (hipMalloc((void **)&dev, kBytes) != hipSuccess) {
            (void)hipGetLastError();
            dev = nullptr;
            return false;
        }
        return true;
    }
    void release() {
        for (int k = 0; k < 2; ++k) {
            if (ev[k]) (void)hipEventSynchronize(ev[k]), (void)hipEventDestroy(ev[k]);
            if (buf[k]) (void)hipHostFree(buf[k]);
            ev[k] = nullptr;
            buf[k] = nullptr;
        }
        if (dev) (void)hipFree(dev);
        dev = nullptr;
    }
    // host -> device on stream st; returns once the last chunk is queued
    // (the buffers stay in use until their events complete)
    void upload(void *dst, const void *src, size_t bytes, hipStream_t st) {
        for (size_t off = 0; off < bytes; off += kBytes) {
            const size_t n = std::min(kBytes, bytes - off);
            const int k = next;
            next ^= 1;
            DF_HIP(hipEventSynchronize(ev[k]));  // the buffer's previous copy is done
            std::memcpy(buf[k], (const char *)src + off, n);
            DF_HIP(hipMemcpyAsync((char *)dst + off, buf[k], n, hipMemcpyHostToDevice, st));
            DF_HIP(hipEventRecord(ev[k], st));
        }
    }
    // device -> host on stream st, waiting for the copies (the host copy of
    // one chunk overlaps the device copy of the next)
    void download(void *dst, const void *src, size_t bytes, hipStream_t st) {
        size_t pend_off = 0, pend_n = 0;
        int pend_k = -1;
        auto drain = [&] {
            if (pend_k < 0) return;
            DF_HIP(hipEventSynchronize(ev[pend_k]));
            std::memcpy((char *)dst + pend_off, buf[pend_k], pend_n);
            pend_k = -1;
        };
        for (size_t off = 0; off < bytes; off += kBytes) {
            const size_t n = std::min(kBytes, bytes - off);
            const int k = next;
            next ^= 1;
            DF_HIP(hipEventSynchronize(ev[k]));
            DF_HIP(hipMemcpyAsync(buf[k], (const char *)src + off, n, hipMemcpyDeviceToHost, st));
            DF_HIP(hipEventRecord(ev[k], st));
            drain();
            pend_off = off, pend_n = n, pend_k = k;
        }
        drain();
    }
    // host FP32 -> device BF16 (rounded on the device), on stream st: each
    // chunk is copied into the device buffer and rounded from there (stream
    // order keeps the next chunk's copy behind the rounding)
    void upload_bf16(uint16_t *dst, const float *src, size_t count, hipStream_t st) {
        constexpr size_t per = kBytes / 4;
        for (size_t off = 0; off < count; off += per) {
            const size_t n = std::min(per, count - off);
            const int k = next;
            next ^= 1;
            DF_HIP(hipEventSynchronize(ev[k]));
            std::memcpy(buf[k], src + off, 4 * n);
            DF_HIP(hipMemcpyAsync(dev, buf[k], 4 * n, hipMemcpyHostToDevice, st));
            DF_HIP(hipEventRecord(ev[k], st));
            hipLaunchKernelGGL(k_f32_to_bf16, dim3(convert_grid((int64_t)n)), dim3(256), 0, st,
                               (const float *)dev, dst + off, (int64_t)n);
            DF_LAUNCHED();
        }
    }
    // device BF16 -> host FP32 (widened on the device), on stream st, waiting
    // for the copies
    void download_bf16(float *dst, const uint16_t *src, size_t count, hipStream_t st) {
        constexpr size_t per = kBytes / 4;
        size_t pend_off = 0, pend_n = 0;
        int pend_k = -1;
        auto drain = [&] {
            if (pend_k < 0) return;
            DF_HIP(hipEventSynchronize(ev[pend_k]));
            std::memcpy(dst + pend_off, buf[pend_k], 4 * pend_n);
            pend_k = -1;
        };
        for (size_t off = 0; off < count; off += per) {
            const size_t n = std::min(per, count - off);
            const int k = next;
            next ^= 1;
            DF_HIP(hipEventSynchronize(ev[k]));
            hipLaunchKernelGGL(k_bf16_to_f32, dim3(convert_grid((int64_t)n)), dim3(256), 0, st,
                               src + off, dev, (int64_t)n);
            DF_LAUNCHED();
            DF_HIP(hipMemcpyAsync(buf[k], dev, 4 * n, hipMemcpyDeviceToHost, st));
            DF_HIP(hipEventRecord(ev[k], st));
            drain();
            pend_off = off, pend_n = n, pend_k = k;
        }
        drain();
    }
};

}  // namespace

struct dfacto_server {
    int device = 0;
    size_t budget = 0;
    int max_slots = 1;
    dfacto_ctx *ctx = nullptr;  // the worker's context (own stream)
    hipStream_t stream = nullptr;
    hipStream_t dstream = nullptr;  // the delivery thread's stream
    // the server's own pool for every stream-ordered allocation it makes; it
    // keeps freed memory mapped (the default pool unmaps it at each
    // synchronization, which made a long-running server progressively slower)
    hipMemPool_t pool = nullptr;
    static constexpr int kBuilders = 2;
    dfacto_ctx *bctx[kBuilders] = {};  // the builders' contexts (own streams)
    hipStream_t bstream[kBuilders] = {};
    Staging bstage[kBuilders], dstage;  // pinned staging: builders, delivery
    Clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv_work, cv_build, cv_deliver, cv_done;
    bool stop = false;
    int64_t next_id = 1;
    std::deque<std::unique_ptr<Member>> pending;  // submitted, not yet admitted
    std::deque<std::unique_ptr<Member>> ready;    // built, not yet attached
    std::deque<std::unique_ptr<Member>> retired;  // stopped, results not yet delivered
    bool worker_done = false;
    std::map<int64_t, dfacto_request_status> finished;  // id -> final status
    std::map<int64_t, int> running;                     // ids admitted and not yet done
    int slots = 0;     // requests admitted and not yet retired (building, ready or active)
    size_t used = 0;   // device bytes reserved by those requests
    int peak_active = 0;
    int64_t iterations = 0;
    double t_admit = 0, t_build = 0, t_groups = 0, t_iterate = 0, t_deliver = 0;

    // worker-only state
    std::vector<std::unique_ptr<Member>> active;
    std::vector<dfacto_group *> groups;  // over `active`, rebuilt when it changes
    bool dirty = true;
    double *d_fits = nullptr;  // max_slots doubles
    std::thread worker, deliverer, builder[kBuilders];
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

// Peak transient device memory of building the flattenings: COO staging,
// sort keys and permutations, gathered copies (about 80 bytes per nonzero
// with buffers reused within the build), plus the build's arena of small
// temporaries, which are kept until the build ends (at most about 160 bytes
// per nonzero and 24 per row, doubled for chunk rounding, and at most a
// few chunks of up to 1 GB).
size_t build_transient(const dfacto_request &r) {
    const size_t rows = (size_t)(r.dims[0] + r.dims[1] + r.dims[2]);
    const size_t arena = std::min<size_t>(320 * (size_t)r.nnz + 48 * rows + (32 << 20),
                                          (size_t)1 << 30);
    return 80 * (size_t)r.nnz + arena + (1 << 20);
}

// Release a member's memory, ordered on the stream it was allocated on.  The
// caller has already waited for every kernel that reads it.
void free_member(Member &m) {
    for (int k = 0; k < 3; ++k)
        if (m.F[k]) (void)hipFreeAsync(m.F[k], m.mem_stream), m.F[k] = nullptr;
    if (m.lambda) (void)hipFreeAsync(m.lambda, m.mem_stream), m.lambda = nullptr;
    if (m.tensor) dfacto_tensor_destroy(m.tensor), m.tensor = nullptr;
}

// Record a request's final status and give back its slot and bytes.
void finish(dfacto_server *s, std::unique_ptr<Member> mp, dfacto_status status) {
    Member &m = *mp;
    m.st.status = status;
    m.st.done = 1;
    m.st.t_done = seconds_since(s, Clock::now());
    std::lock_guard<std::mutex> lk(s->mu);
    s->running.erase(m.id);
    s->finished[m.id] = m.st;
    s->slots -= 1;
    s->used -= std::min(s->used, m.footprint);
    s->cv_done.notify_all();
    s->cv_build.notify_one();
    s->cv_work.notify_one();
}

// Upload, build and initialize one request on builder b's stream; all of
// its memory is stream-ordered on that stream.  Returns after the stream has
// finished, so the member is ready for kernels on any stream.  *t_build
// receives the time of the flattening build.
void admit(dfacto_server *s, int b, Member &m, double *t_build) {
    const dfacto_request &r = m.req;
    hipStream_t st = s->bstream[b];
    m.mem_stream = st;
    uint32_t *di = nullptr, *dj = nullptr, *dk = nullptr;
    float *dv = nullptr;
    const size_t n = (size_t)std::max<int64_t>(r.nnz, 1);
    auto cleanup = [&] {  // stream-ordered: no wait for the other requests' work
        if (di) (void)hipFreeAsync(di, st);
        if (dj) (void)hipFreeAsync(dj, st);
        if (dk) (void)hipFreeAsync(dk, st);
        if (dv) (void)hipFreeAsync(dv, st);
    };
    try {
        hip_check(stream_alloc((void **)&di, 4 * n, st, s->pool), "request upload");
        hip_check(stream_alloc((void **)&dj, 4 * n, st, s->pool), "request upload");
        hip_check(stream_alloc((void **)&dk, 4 * n, st, s->pool), "request upload");
        hip_check(stream_alloc((void **)&dv, 4 * n, st, s->pool), "request upload");
        Staging &sg = s->bstage[b];
        if (r.nnz > 0) {
            sg.upload(di, r.i, 4 * r.nnz, st);
            sg.upload(dj, r.j, 4 * r.nnz, st);
            sg.upload(dk, r.k, 4 * r.nnz, st);
            sg.upload(dv, r.val, 4 * r.nnz, st);
        }
        const auto tb = Clock::now();
        const dfacto_status bs =
            build_flattenings_async_alloc(s->bctx[b], r.dims, r.nnz, di, dj, dk, dv, &m.tensor);
        *t_build = std::chrono::duration<double>(Clock::now() - tb).count();
        if (bs != DFACTO_OK) throw Error{bs, dfacto_last_error(s->bctx[b])};
        cleanup();
        di = dj = dk = nullptr;
        dv = nullptr;
        const size_t es = r.dtype == DFACTO_BF16 ? 2 : 4;
        for (int k = 0; k < 3; ++k) {
            const size_t cnt = (size_t)r.dims[k] * r.R;
            hip_check(stream_alloc(&m.F[k], std::max<size_t>(es * cnt, 16), st, s->pool),
                      "factor allocation");
            if (r.dtype == DFACTO_BF16) {  // FP32 upload, rounded to BF16 on the device
                sg.upload_bf16((uint16_t *)m.F[k], r.init[k], cnt, st);
            } else {
                sg.upload(m.F[k], r.init[k], 4 * cnt, st);
            }
        }
        hip_check(stream_alloc((void **)&m.lambda, 8 * (size_t)r.R, st, s->pool),
                  "lambda allocation");
        DF_HIP(hipStreamSynchronize(st));
        m.footprint = std::max(m.footprint, m.tensor->bytes + footprint_estimate(r) -
                                                3 * 16 * (size_t)r.nnz);
    } catch (...) {
        cleanup();
        (void)hipStreamSynchronize(st);
        throw;
    }
}

// Copy a finished request's factors (BF16 widened to FP32 on the device) and
// lambda to its host buffers, on the delivery stream.
void deliver(dfacto_server *s, Member &m) {
    const dfacto_request &r = m.req;
    hipStream_t st = s->dstream;
    Staging &sg = s->dstage;
    try {
        for (int k = 0; k < 3; ++k) {
            const size_t cnt = (size_t)r.dims[k] * r.R;
            if (!r.out_F[k]) continue;
            if (r.dtype == DFACTO_BF16)
                sg.download_bf16(r.out_F[k], (const uint16_t *)m.F[k], cnt, st);
            else
                sg.download(r.out_F[k], m.F[k], 4 * cnt, st);
        }
        if (r.out_lambda) sg.download(r.out_lambda, m.lambda, 8 * (size_t)r.R, st);
        DF_HIP(hipStreamSynchronize(st));
    } catch (...) {
        (void)hipStreamSynchronize(st);
        throw;
    }
}

void drop_groups(dfacto_server *s) {
    for (dfacto_group *g : s->groups) dfacto_group_destroy(g);
    s->groups.clear();
    s->dirty = true;
}

// Groups over the active requests.  The active list is kept ordered by
// (dtype, reg); each run of one class is one group, and a class's members
// own consecutive fit slots.  The groups are rebuilt only when the active
// set changes.
void build_groups(dfacto_server *s) {
    {
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
                                    lam.data(), s->d_fits + a,
                                    DFACTO_GROUP_CTX_STREAM | DFACTO_GROUP_OWN_FACTORS, &g);
            if (st != DFACTO_OK) throw Error{st, dfacto_last_error(s->ctx)};
            s->groups.push_back(g);
            a = b;
        }
        s->dirty = false;
    }
}

// Whether the next queued request can be admitted now: a slot is free and
// its footprint fits the budget.  A request is always admitted when nothing
// else holds a slot (it fails with E_NOMEM if the device cannot hold it).
bool can_admit(const dfacto_server *s) {
    if (s->pending.empty() || s->slots >= s->max_slots) return false;
    const dfacto_request &r = s->pending.front()->req;
    return s->slots == 0 || s->used + footprint_estimate(r) + build_transient(r) <= s->budget;
}

void builder_main(dfacto_server *s, int b) {
    (void)hipSetDevice(s->device);
    for (;;) {
        std::unique_ptr<Member> m;
        size_t reserved = 0;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_build.wait(lk, [&] { return (s->stop && s->pending.empty()) || can_admit(s); });
            if (s->pending.empty()) return;  // stopping, nothing left to admit
            m = std::move(s->pending.front());
            s->pending.pop_front();
            reserved = footprint_estimate(m->req) + build_transient(m->req);
            m->footprint = reserved;
            s->running[m->id] = 1;
            s->slots += 1;
            s->used += reserved;
            m->st.t_admit = seconds_since(s, Clock::now());  // in arrival order
        }
        const auto ta = Clock::now();
        dfacto_status code = DFACTO_OK;
        double tbuild = 0;
        try {
            admit(s, b, *m, &tbuild);
        } catch (const Error &e) {
            code = e.code;
        }
        const double dt = std::chrono::duration<double>(Clock::now() - ta).count();
        if (code != DFACTO_OK) {
            free_member(*m);
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->t_admit += dt;
                s->t_build += tbuild;
            }
            finish(s, std::move(m), code);
            continue;
        }
        // the reservation shrinks to what the built request holds
        const size_t held = std::max(m->tensor->bytes + footprint_estimate(m->req) -
                                         std::min(footprint_estimate(m->req), 3 * 16 * (size_t)m->req.nnz),
                                     footprint_estimate(m->req));
        std::lock_guard<std::mutex> lk(s->mu);
        s->t_admit += dt;
        s->t_build += tbuild;
        s->used = s->used - std::min(s->used, reserved) + held;
        m->footprint = held;
        s->ready.push_back(std::move(m));
        s->cv_work.notify_one();
        s->cv_build.notify_one();
    }
}

void deliverer_main(dfacto_server *s) {
    (void)hipSetDevice(s->device);
    for (;;) {
        std::unique_ptr<Member> m;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_deliver.wait(lk, [&] { return !s->retired.empty() || s->worker_done; });
            if (s->retired.empty()) return;  // the worker has ended and nothing is left
            m = std::move(s->retired.front());
            s->retired.pop_front();
        }
        dfacto_status code = DFACTO_OK;
        const auto td = Clock::now();
        try {
            deliver(s, *m);
        } catch (const Error &e) {
            code = e.code;
        }
        free_member(*m);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->t_deliver += std::chrono::duration<double>(Clock::now() - td).count();
        }
        finish(s, std::move(m), code);
    }
}

void worker_main(dfacto_server *s) {
    (void)hipSetDevice(s->device);
    std::deque<std::unique_ptr<Member>> arrived;
    for (;;) {
        // attach the built requests
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] {
                return (s->stop && s->pending.empty() && s->slots == 0) || !s->ready.empty() ||
                       !s->active.empty();
            });
            if (s->active.empty() && s->ready.empty()) {  // stopping, all done
                s->worker_done = true;
                s->cv_deliver.notify_all();
                return;
            }
            arrived.swap(s->ready);
        }
        if (!arrived.empty()) {
            drop_groups(s);  // the groups refer to the old active set
            for (auto &m : arrived) s->active.push_back(std::move(m));
            arrived.clear();
            std::lock_guard<std::mutex> lk(s->mu);
            s->peak_active = std::max(s->peak_active, (int)s->active.size());
        }
        // one iteration for everyone, then the stopping rule per request
        try {
            const auto ti = Clock::now();
            double tg = 0;
            {
                const auto tg0 = Clock::now();
                if (s->dirty) build_groups(s);
                tg = std::chrono::duration<double>(Clock::now() - tg0).count();
            }
            for (dfacto_group *g : s->groups) {
                const dfacto_status st = dfacto_group_als(s->ctx, g, 1);
                if (st != DFACTO_OK) throw Error{st, dfacto_last_error(s->ctx)};
            }
            std::vector<double> fits(s->active.size());
            DF_HIP(hipMemcpyAsync(fits.data(), s->d_fits, 8 * fits.size(), hipMemcpyDeviceToHost,
                                  s->stream));
            DF_HIP(hipStreamSynchronize(s->stream));
            const double titer = std::chrono::duration<double>(Clock::now() - ti).count() - tg;
            std::vector<std::unique_ptr<Member>> keep, done;
            for (size_t a = 0; a < s->active.size(); ++a) {
                std::unique_ptr<Member> &m = s->active[a];
                m->st.iters += 1;
                m->st.fit = fits[a];
                const bool conv = m->has_prev && std::fabs(fits[a] - m->prev_fit) < m->req.tol;
                m->prev_fit = fits[a];
                m->has_prev = true;
                if (conv || m->st.iters >= m->req.max_iters) {
                    // the groups read its memory: drop them before delivery frees it
                    if (!s->groups.empty()) drop_groups(s);
                    done.push_back(std::move(m));
                } else {
                    keep.push_back(std::move(m));
                }
            }
            s->active.swap(keep);
            std::lock_guard<std::mutex> lk(s->mu);
            for (auto &m : done) s->retired.push_back(std::move(m));
            done.clear();
            if (!s->retired.empty()) s->cv_deliver.notify_one();
            ++s->iterations;
            s->t_groups += tg;
            s->t_iterate += titer;
        } catch (const Error &e) {
            // a device failure ends every active request with its code
            drop_groups(s);
            for (auto &m : s->active) {
                free_member(*m);
                finish(s, std::move(m), e.code);
            }
            s->active.clear();
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
    if (hipStreamCreateWithFlags(&s->dstream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipStreamDestroy(s->stream);
        delete s;
        return DFACTO_E_DEVICE;
    }
    for (int b = 0; b < dfacto_server::kBuilders; ++b)
        if (hipStreamCreateWithFlags(&s->bstream[b], hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            for (int c = 0; c < b; ++c) (void)hipStreamDestroy(s->bstream[c]);
            (void)hipStreamDestroy(s->dstream);
            (void)hipStreamDestroy(s->stream);
            delete s;
            return DFACTO_E_DEVICE;
        }
    {
        hipMemPoolProps props{};
        props.allocType = hipMemAllocationTypePinned;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = device;
        uint64_t keep = UINT64_MAX;
        if (hipMemPoolCreate(&s->pool, &props) != hipSuccess ||
            hipMemPoolSetAttribute(s->pool, hipMemPoolAttrReleaseThreshold, &keep) != hipSuccess) {
            (void)hipGetLastError();
            if (s->pool) (void)hipMemPoolDestroy(s->pool);
            for (int b = 0; b < dfacto_server::kBuilders; ++b) (void)hipStreamDestroy(s->bstream[b]);
            (void)hipStreamDestroy(s->dstream);
            (void)hipStreamDestroy(s->stream);
            delete s;
            return DFACTO_E_DEVICE;
        }
    }
    if (hbm_budget == 0) {  // default: 90% of the free device memory
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess) hbm_budget = fr / 10 * 9;
    }
    s->budget = hbm_budget;
    bool ok = hipMalloc(&s->d_fits, 8 * (size_t)max_slots) == hipSuccess &&
              dfacto_ctx_create(device, s->stream, nullptr, &s->ctx) == DFACTO_OK;
    for (int b = 0; ok && b < dfacto_server::kBuilders; ++b)
        ok = dfacto_ctx_create(device, s->bstream[b], nullptr, &s->bctx[b]) == DFACTO_OK;
    for (int b = 0; ok && b < dfacto_server::kBuilders; ++b) ok = s->bstage[b].init();
    ok = ok && s->dstage.init();
    if (ok) {
        s->ctx->mem.pool = s->pool;
        for (int b = 0; b < dfacto_server::kBuilders; ++b) s->bctx[b]->mem.pool = s->pool;
    }
    if (!ok) {
        (void)hipGetLastError();
        for (int b = 0; b < dfacto_server::kBuilders; ++b) s->bstage[b].release();
        s->dstage.release();
        if (s->ctx) dfacto_ctx_destroy(s->ctx);
        for (int b = 0; b < dfacto_server::kBuilders; ++b) {
            if (s->bctx[b]) dfacto_ctx_destroy(s->bctx[b]);
            (void)hipStreamDestroy(s->bstream[b]);
        }
        if (s->d_fits) (void)hipFree(s->d_fits);
        (void)hipMemPoolDestroy(s->pool);
        (void)hipStreamDestroy(s->dstream);
        (void)hipStreamDestroy(s->stream);
        delete s;
        return DFACTO_E_DEVICE;
    }
    if (prev >= 0) (void)hipSetDevice(prev);
    s->worker = std::thread(worker_main, s);
    s->deliverer = std::thread(deliverer_main, s);
    for (int b = 0; b < dfacto_server::kBuilders; ++b) s->builder[b] = std::thread(builder_main, s, b);
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
    s->cv_build.notify_one();
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
    out->t_admit = s->t_admit;
    out->t_build = s->t_build;
    out->t_groups = s->t_groups;
    out->t_iterate = s->t_iterate;
    out->t_deliver = s->t_deliver;
    return DFACTO_OK;
}

void dfacto_server_destroy(dfacto_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    s->cv_build.notify_all();
    for (auto &b : s->builder)
        if (b.joinable()) b.join();
    if (s->worker.joinable()) s->worker.join();
    if (s->deliverer.joinable()) s->deliverer.join();
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    drop_groups(s);
    for (auto &m : s->active) free_member(*m);
    if (s->ctx) dfacto_ctx_destroy(s->ctx);
    if (s->d_fits) (void)hipFree(s->d_fits);
    for (int b = 0; b < dfacto_server::kBuilders; ++b) {
        if (s->bctx[b]) dfacto_ctx_destroy(s->bctx[b]);
        (void)hipStreamSynchronize(s->bstream[b]);  // stream-ordered frees
        (void)hipStreamDestroy(s->bstream[b]);
    }
    for (int b = 0; b < dfacto_server::kBuilders; ++b) s->bstage[b].release();
    s->dstage.release();
    if (s->dstream) (void)hipStreamDestroy(s->dstream);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    // every allocation from the pool has been freed and its stream finished
    (void)hipDeviceSynchronize();
    if (s->pool) (void)hipMemPoolDestroy(s->pool);
    if (prev >= 0) (void)hipSetDevice(prev);
    delete s;
}

}  // extern "C"
