// Serving runtime of lbessel: FIFO admission into a device arena by memory,
// continuous batching of evaluation requests into segmented launches, vMF
// fits on the device, several batches in flight on separate streams.  The
// request flow and the guarantees are described in include/lbessel_serve.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lbessel.h"
#include "lbessel_serve.h"

namespace {

using Clock = std::chrono::steady_clock;

constexpr int64_t kAlign = 256;
constexpr int kGroups = 4;          // (kind, precision): I64, K64, I32, K32
constexpr int64_t kVmfResult = 256; // arena bytes reserved for the 4 result doubles

int64_t align_up(int64_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, total) with coalescing of neighbours.
class Arena {
  public:
    explicit Arena(int64_t total) : total_(total) { free_[0] = total; }

    int64_t alloc(int64_t size) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < size)
                continue;
            const int64_t off = it->first, rest = it->second - size;
            free_.erase(it);
            if (rest > 0)
                free_[off + size] = rest;
            used_ += size;
            peak_ = std::max(peak_, used_);
            return off;
        }
        return -1;
    }

    void release(int64_t off, int64_t size) {
        used_ -= size;
        auto it = free_.emplace(off, size).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

    int64_t total() const { return total_; }
    int64_t peak() const { return peak_; }

  private:
    std::map<int64_t, int64_t> free_;   // offset -> size
    int64_t total_, used_ = 0, peak_ = 0;
};

enum ReqType { REQ_EVAL = 0, REQ_VMF = 1, REQ_EVAL_DEVICE = 2 };

struct Request {
    int64_t id = 0;
    int type = REQ_EVAL;
    int kind = 0, precision = 64;
    const void *hv = nullptr, *hx = nullptr;
    void *hout = nullptr;
    int64_t n = 0;
    const float *X = nullptr;
    int64_t p = 0;
    double *hres = nullptr;
    int64_t off = -1;
    bool dev = false;   // evaluation arrays in device memory: no copies, no arena data
    lbessel_request_info_t info{};

    int group() const { return (precision == 64 ? 0 : 2) + kind; }
    int64_t elem() const { return precision == 64 ? 8 : 4; }
    int64_t span() const { return align_up(n * elem()); }   // one array in the arena
};

// One stream with the batch it runs.  Every request of the batch gets its own
// completion event, recorded right after its result copy, so it completes as
// soon as its own outputs are back rather than with the whole batch; events
// on one stream complete in the order they were recorded.
struct Slot {
    hipStream_t stream = nullptr;
    std::vector<hipEvent_t> ev;          // one per request of a batch
    lbessel_segment_t *hseg = nullptr;   // pinned staging, kGroups * cap entries
    lbessel_segment_t *dseg = nullptr;   // device copy
    std::vector<Request *> reqs;         // the batch
    std::vector<Request *> order;        // requests in event-record order
    size_t next_done = 0;                // first entry of order not yet complete
    bool busy = false;
};

double seconds_since(Clock::time_point t0) {
    return std::chrono::duration<double>(Clock::now() - t0).count();
}

}  // namespace

struct lbessel_server {
    lbessel_server_config_t cfg{};
    int device = 0;
    char *arena_dev = nullptr;
    std::unique_ptr<Arena> arena;
    std::vector<Slot> slots;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;      // submitted, waiting for admission (FIFO)
    std::deque<Request *> admitted;   // holding arena memory, not yet launched
    std::unordered_map<int64_t, std::unique_ptr<Request>> live;
    int64_t next_id = 1;
    int64_t next_batch = 0;
    bool stopping = false;
    lbessel_server_stats_t stats{};
    std::thread worker;
    Clock::time_point t0 = Clock::now();

    double now() const { return seconds_since(t0); }
    int64_t bytes_of(const Request &r) const;
    int enqueue(Slot &sl, int64_t *launches);
    void run();
    int submit(std::unique_ptr<Request> r, int64_t *ticket);
};

int64_t lbessel_server::bytes_of(const Request &r) const {
    if (r.type == REQ_EVAL)
        return r.dev ? kAlign : std::max<int64_t>(kAlign, 3 * r.span());   // v, x, out
    const int64_t w = lbessel_vmf_fit_workspace(r.n, r.p);
    return (w < 0) ? -1 : kVmfResult + align_up(w);
}

// Enqueue one batch on its stream (no lock held).  Records the slot's event
// even after an error, so the batch always completes.  *launches receives
// the number of evaluation kernels launched.
int lbessel_server::enqueue(Slot &sl, int64_t *launches) {
    *launches = 0;
    hipStream_t st = sl.stream;
    int rc = LBESSEL_OK;
    auto keep = [&rc](int r) {
        if (rc == LBESSEL_OK && r != LBESSEL_OK)
            rc = r;
    };
    auto hip = [&keep](hipError_t e) { keep(e == hipSuccess ? LBESSEL_OK : LBESSEL_EHIP); };
    const bool plain = (cfg.mode == LBESSEL_SERVE_PLAIN);
    const int cap = cfg.max_batch_requests;

    // vMF fits first: their inputs are already on the device.
    for (Request *r : sl.reqs) {
        if (r->type != REQ_VMF)
            continue;
        double *res = reinterpret_cast<double *>(arena_dev + r->off);
        char *work = arena_dev + r->off + kVmfResult;
        keep(lbessel_vmf_fit_f32(r->X, r->n, r->p, res, work, r->info.bytes - kVmfResult, st));
        hip(hipMemcpyAsync(r->hres, res, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
        hip(hipEventRecord(sl.ev[sl.order.size()], st));
        sl.order.push_back(r);
    }
    // Evaluation requests, one group per (kind, precision).
    for (int g = 0; g < kGroups; ++g) {
        const int kind = g & 1, prec = (g < 2) ? 64 : 32;
        int count = 0;
        int64_t tiles = 0;
        lbessel_segment_t *hs = sl.hseg + int64_t(g) * cap;
        for (Request *r : sl.reqs) {
            if (r->type != REQ_EVAL || r->group() != g)
                continue;
            char *dv = r->dev ? (char *)r->hv : arena_dev + r->off;
            char *dx = r->dev ? (char *)r->hx : dv + r->span();
            char *dout = r->dev ? (char *)r->hout : dx + r->span();
            const int64_t nb = r->n * r->elem();
            if (nb > 0 && !r->dev) {
                hip(hipMemcpyAsync(dv, r->hv, nb, hipMemcpyHostToDevice, st));
                hip(hipMemcpyAsync(dx, r->hx, nb, hipMemcpyHostToDevice, st));
            }
            if (plain) {
                int e;
                if (prec == 64)
                    e = (kind == 0) ? lbessel_log_iv_f64((const double *)dv, (const double *)dx,
                                                         (double *)dout, r->n, st)
                                    : lbessel_log_kv_f64((const double *)dv, (const double *)dx,
                                                         (double *)dout, r->n, st);
                else
                    e = (kind == 0) ? lbessel_log_iv_f32((const float *)dv, (const float *)dx,
                                                         (float *)dout, r->n, st)
                                    : lbessel_log_kv_f32((const float *)dv, (const float *)dx,
                                                         (float *)dout, r->n, st);
                keep(e);
                if (r->n > 0)
                    ++*launches;
            } else if (r->n > 0) {
                hs[count++] = lbessel_segment_t{dv, dx, dout, r->n, tiles};
                tiles += lbessel_segment_tiles(r->n);
            }
        }
        if (!plain && tiles > 0) {
            if (count <= LBESSEL_SEG_INLINE_MAX) {
                // small batch: the table rides in the kernel arguments
                keep(lbessel_eval_segments_inline(kind, prec, hs, count, tiles, st));
            } else {
                lbessel_segment_t *ds = sl.dseg + int64_t(g) * cap;
                hip(hipMemcpyAsync(ds, hs, count * sizeof(lbessel_segment_t),
                                   hipMemcpyHostToDevice, st));
                keep(lbessel_eval_segments(kind, prec, ds, count, tiles, st));
            }
            ++*launches;
        }
        for (Request *r : sl.reqs) {
            if (r->type != REQ_EVAL || r->group() != g)
                continue;
            if (r->n > 0 && !r->dev) {
                const char *dout = arena_dev + r->off + 2 * r->span();
                hip(hipMemcpyAsync(r->hout, dout, r->n * r->elem(), hipMemcpyDeviceToHost, st));
            }
            hip(hipEventRecord(sl.ev[sl.order.size()], st));
            sl.order.push_back(r);
        }
    }
    return rc;
}

void lbessel_server::run() {
    (void)hipSetDevice(device);   // the device was valid at create
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        bool progress = false;
        int busy = 0;
        // 1. retire finished batches
        for (Slot &sl : slots) {
            if (!sl.busy)
                continue;
            while (sl.next_done < sl.order.size()) {
                const hipError_t e = hipEventQuery(sl.ev[sl.next_done]);
                if (e == hipErrorNotReady)
                    break;
                Request *r = sl.order[sl.next_done++];
                if (e != hipSuccess && r->info.status == LBESSEL_OK)
                    r->info.status = LBESSEL_EHIP;
                r->info.t_done = now();
                r->info.state = LBESSEL_REQ_DONE;
                arena->release(r->off, r->info.bytes);
                ++stats.completed;
                if (r->type == REQ_EVAL)
                    stats.eval_pairs += r->n;
                else
                    ++stats.vmf_fits;
                progress = true;
            }
            if (sl.next_done == sl.order.size()) {
                sl.reqs.clear();
                sl.order.clear();
                sl.next_done = 0;
                sl.busy = false;
            } else {
                ++busy;
            }
        }
        if (progress)
            cv_done.notify_all();
        // 2. admission by memory, strictly FIFO
        while (!queue.empty()) {
            Request *r = queue.front();
            const int64_t off = arena->alloc(r->info.bytes);
            if (off < 0)
                break;
            r->off = off;
            r->info.t_admit = now();
            r->info.state = LBESSEL_REQ_ADMITTED;
            admitted.push_back(r);
            queue.pop_front();
            progress = true;
        }
        stats.arena_peak_bytes = arena->peak();
        // 3. launch the next batch on a free stream
        Slot *free_slot = nullptr;
        for (Slot &sl : slots)
            if (!sl.busy) {
                free_slot = &sl;
                break;
            }
        if (free_slot != nullptr && !admitted.empty()) {
            Slot &sl = *free_slot;
            int64_t elems = 0;
            const size_t max_req =
                (cfg.mode == LBESSEL_SERVE_PLAIN) ? 1 : size_t(cfg.max_batch_requests);
            while (!admitted.empty() && sl.reqs.size() < max_req) {
                Request *r = admitted.front();
                const int64_t add = (r->type == REQ_EVAL) ? r->n : 0;
                const bool solo = (r->type != REQ_EVAL) || add >= cfg.solo_elems;
                if (!sl.reqs.empty() && (solo || elems + add > cfg.max_batch_elems))
                    break;
                elems += add;
                sl.reqs.push_back(r);
                admitted.pop_front();
                if (solo)
                    break;
            }
            const int64_t b = next_batch++;
            const double t = now();
            for (Request *r : sl.reqs) {
                r->info.batch = b;
                r->info.t_launch = t;
                r->info.state = LBESSEL_REQ_LAUNCHED;
            }
            sl.busy = true;
            ++stats.batches;
            stats.max_batch_requests_seen =
                std::max<int64_t>(stats.max_batch_requests_seen, int64_t(sl.reqs.size()));
            lk.unlock();
            int64_t launches = 0;
            const int rc = enqueue(sl, &launches);
            lk.lock();
            stats.kernel_launches += launches;
            if (rc != LBESSEL_OK)
                for (Request *r : sl.reqs)
                    r->info.status = rc;
            if (sl.order.size() != sl.reqs.size()) {
                // an event could not be recorded: finish the batch at once
                // after the stream drains, so no request waits forever
                (void)hipStreamSynchronize(sl.stream);
                sl.order = sl.reqs;
                for (size_t k = 0; k < sl.order.size(); ++k)
                    (void)hipEventRecord(sl.ev[k], sl.stream);
            }
            continue;   // look again at once: more may be launchable
        }
        if (stopping && queue.empty() && admitted.empty() && busy == 0)
            break;
        if (progress)
            continue;
        if (busy > 0) {
            if (cfg.poll_us > 0) {
                cv_work.wait_for(lk, std::chrono::microseconds(cfg.poll_us));
            } else {
                lk.unlock();
                std::this_thread::yield();
                lk.lock();
            }
        } else {
            cv_work.wait(lk, [this] { return stopping || !queue.empty() || !admitted.empty(); });
        }
    }
}

int lbessel_server::submit(std::unique_ptr<Request> r, int64_t *ticket) {
    const int64_t bytes = bytes_of(*r);
    if (bytes < 0)
        return LBESSEL_EINVAL;
    if (bytes > arena->total())
        return LBESSEL_ETOOBIG;
    std::lock_guard<std::mutex> lk(mu);
    if (stopping)
        return LBESSEL_ESTOPPED;
    r->id = next_id++;
    r->info.status = LBESSEL_OK;
    r->info.state = LBESSEL_REQ_QUEUED;
    r->info.batch = -1;
    r->info.bytes = bytes;
    r->info.t_submit = now();
    r->info.t_arrival = r->info.t_submit;
    Request *raw = r.get();
    live.emplace(raw->id, std::move(r));
    queue.push_back(raw);
    ++stats.submitted;
    stats.queue_peak = std::max<int64_t>(stats.queue_peak, int64_t(queue.size()));
    if (ticket != nullptr)
        *ticket = raw->id;
    cv_work.notify_one();
    return LBESSEL_OK;
}

extern "C" {

void lbessel_server_default_config(lbessel_server_config_t *cfg) {
    if (cfg == nullptr)
        return;
    cfg->arena_bytes = int64_t(2) << 30;
    cfg->streams = 8;
    cfg->mode = LBESSEL_SERVE_BATCHED;
    cfg->max_batch_requests = 64;
    cfg->max_batch_elems = int64_t(1) << 18;
    cfg->poll_us = 0;
    cfg->solo_elems = int64_t(1) << 16;
}

int lbessel_server_create(const lbessel_server_config_t *cfg, lbessel_server_t **out) {
    if (cfg == nullptr || out == nullptr || cfg->arena_bytes <= 0 || cfg->streams < 1 ||
        cfg->streams > 16 || (cfg->mode != LBESSEL_SERVE_BATCHED && cfg->mode != LBESSEL_SERVE_PLAIN) ||
        cfg->max_batch_requests < 1 || cfg->max_batch_requests > 1024 ||
        cfg->max_batch_elems < 1 || cfg->poll_us < 0 || cfg->solo_elems < 1)
        return LBESSEL_EINVAL;
    *out = nullptr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return LBESSEL_ENODEV;
    auto s = std::make_unique<lbessel_server>();
    s->cfg = *cfg;
    s->cfg.arena_bytes = align_up(cfg->arena_bytes);
    s->device = dev;
    if (hipMalloc(reinterpret_cast<void **>(&s->arena_dev), size_t(s->cfg.arena_bytes)) !=
        hipSuccess)
        return LBESSEL_EHIP;
    s->arena = std::make_unique<Arena>(s->cfg.arena_bytes);
    s->slots.resize(size_t(cfg->streams));
    const size_t seg_bytes = size_t(kGroups) * size_t(cfg->max_batch_requests) *
                             sizeof(lbessel_segment_t);
    bool ok = true;
    for (Slot &sl : s->slots) {
        ok = ok && hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess;
        sl.ev.assign(size_t(cfg->max_batch_requests), nullptr);
        for (hipEvent_t &e : sl.ev)
            ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
        ok = ok && hipHostMalloc(reinterpret_cast<void **>(&sl.hseg), seg_bytes,
                                 hipHostMallocDefault) == hipSuccess;
        ok = ok && hipMalloc(reinterpret_cast<void **>(&sl.dseg), seg_bytes) == hipSuccess;
    }
    if (!ok) {
        for (Slot &sl : s->slots) {
            if (sl.dseg) (void)hipFree(sl.dseg);
            if (sl.hseg) (void)hipHostFree(sl.hseg);
            for (hipEvent_t e : sl.ev)
                if (e) (void)hipEventDestroy(e);
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
        }
        (void)hipFree(s->arena_dev);
        return LBESSEL_EHIP;
    }
    s->stats.arena_bytes = s->cfg.arena_bytes;
    lbessel_server *raw = s.release();
    raw->worker = std::thread([raw] { raw->run(); });
    *out = raw;
    return LBESSEL_OK;
}

int lbessel_server_submit_eval(lbessel_server_t *s, int kind, int precision, const void *v,
                               const void *x, void *out, int64_t n, int64_t *ticket) {
    if (s == nullptr || (kind != 0 && kind != 1) || (precision != 64 && precision != 32) ||
        n < 0 || (n > 0 && (v == nullptr || x == nullptr || out == nullptr)))
        return LBESSEL_EINVAL;
    auto r = std::make_unique<Request>();
    r->type = REQ_EVAL;
    r->kind = kind;
    r->precision = precision;
    r->hv = v;
    r->hx = x;
    r->hout = out;
    r->n = n;
    return s->submit(std::move(r), ticket);
}

int lbessel_server_submit_eval_device(lbessel_server_t *s, int kind, int precision,
                                      const void *v, const void *x, void *out, int64_t n,
                                      int64_t *ticket) {
    if (s == nullptr || (kind != 0 && kind != 1) || (precision != 64 && precision != 32) ||
        n < 0 || (n > 0 && (v == nullptr || x == nullptr || out == nullptr)))
        return LBESSEL_EINVAL;
    auto r = std::make_unique<Request>();
    r->type = REQ_EVAL;
    r->dev = true;
    r->kind = kind;
    r->precision = precision;
    r->hv = v;
    r->hx = x;
    r->hout = out;
    r->n = n;
    return s->submit(std::move(r), ticket);
}

int lbessel_server_submit_vmf(lbessel_server_t *s, const float *X, int64_t n, int64_t p,
                              double *result, int64_t *ticket) {
    if (s == nullptr || X == nullptr || result == nullptr || n < 1 || n > int64_t(0x7fffffff) ||
        p < 2)
        return LBESSEL_EINVAL;
    auto r = std::make_unique<Request>();
    r->type = REQ_VMF;
    r->X = X;
    r->n = n;
    r->p = p;
    r->hres = result;
    return s->submit(std::move(r), ticket);
}

int lbessel_server_wait(lbessel_server_t *s, int64_t ticket, double timeout_s,
                        lbessel_request_info_t *info) {
    if (s == nullptr)
        return LBESSEL_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->live.find(ticket);
    if (it == s->live.end())
        return LBESSEL_EINVAL;
    Request *r = it->second.get();
    auto done = [r] { return r->info.state == LBESSEL_REQ_DONE; };
    if (timeout_s < 0) {
        s->cv_done.wait(lk, done);
    } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done)) {
        if (info != nullptr)
            *info = r->info;
        return LBESSEL_ETIMEOUT;
    }
    if (info != nullptr)
        *info = r->info;
    const int status = r->info.status;
    s->live.erase(it);
    return status;
}

double lbessel_server_clock(lbessel_server_t *s) { return (s == nullptr) ? -1.0 : s->now(); }

int lbessel_server_stats(lbessel_server_t *s, lbessel_server_stats_t *st) {
    if (s == nullptr || st == nullptr)
        return LBESSEL_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *st = s->stats;
    return LBESSEL_OK;
}

int lbessel_server_destroy(lbessel_server_t *s) {
    if (s == nullptr)
        return LBESSEL_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable())
        s->worker.join();
    (void)hipSetDevice(s->device);
    for (Slot &sl : s->slots) {
        (void)hipStreamSynchronize(sl.stream);
        (void)hipFree(sl.dseg);
        (void)hipHostFree(sl.hseg);
        for (hipEvent_t e : sl.ev)
            (void)hipEventDestroy(e);
        (void)hipStreamDestroy(sl.stream);
    }
    (void)hipFree(s->arena_dev);
    delete s;
    return LBESSEL_OK;
}

int lbessel_server_replay(lbessel_server_t *s, const lbessel_replay_item_t *items, int64_t count,
                          double timeout_s, lbessel_request_info_t *info) {
    if (s == nullptr || count < 0 || (count > 0 && (items == nullptr || info == nullptr)))
        return LBESSEL_EINVAL;
    for (int64_t i = 1; i < count; ++i)
        if (!(items[i].t_arrival >= items[i - 1].t_arrival))
            return LBESSEL_EINVAL;
    std::vector<int64_t> tickets(size_t(count), 0);
    int rc = LBESSEL_OK;
    int64_t submitted = 0;
    const double start = s->now();
    for (int64_t i = 0; i < count; ++i) {
        const lbessel_replay_item_t &it = items[i];
        const double target = start + it.t_arrival;
        // sleep while far from the arrival time, spin for the last 200 us
        for (;;) {
            const double left = target - s->now();
            if (left <= 0)
                break;
            if (left > 2e-4)
                std::this_thread::sleep_for(std::chrono::duration<double>(left - 2e-4));
            else
                std::this_thread::yield();
        }
        int e;
        if (it.type == REQ_EVAL)
            e = lbessel_server_submit_eval(s, it.kind, it.precision, it.v, it.x, it.out, it.n,
                                           &tickets[i]);
        else if (it.type == REQ_EVAL_DEVICE)
            e = lbessel_server_submit_eval_device(s, it.kind, it.precision, it.v, it.x, it.out,
                                                  it.n, &tickets[i]);
        else if (it.type == REQ_VMF)
            e = lbessel_server_submit_vmf(s, it.X, it.n, it.p, it.result, &tickets[i]);
        else
            e = LBESSEL_EINVAL;
        if (e != LBESSEL_OK) {
            rc = e;
            break;
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            auto f = s->live.find(tickets[i]);
            if (f != s->live.end())
                f->second->info.t_arrival = target;
        }
        ++submitted;
    }
    const auto deadline = Clock::now() + std::chrono::duration<double>(timeout_s < 0 ? 1e9 : timeout_s);
    for (int64_t i = 0; i < submitted; ++i) {
        const double left = std::chrono::duration<double>(deadline - Clock::now()).count();
        const int e = lbessel_server_wait(s, tickets[i], std::max(left, 0.0), &info[i]);
        if (e != LBESSEL_OK && rc == LBESSEL_OK)
            rc = e;
    }
    return rc;
}

}  // extern "C"
