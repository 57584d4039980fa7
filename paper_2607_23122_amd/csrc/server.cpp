// Served loop: frame requests against resident scenes, admitted under an HBM
// budget and run concurrently on a pool of stream slots (continuous
// batching).  (Not in the paper, which renders one view per pass.)
//
// The server allocates one device arena of `budget` bytes at creation.  An
// admitted request takes its occluder records (28 B/px), its validation
// workspace (unbiased reuse) and, when the caller gave no output buffer, its
// output (4 B/px) from the arena (first fit, 256-byte aligned); records and
// workspace go back when the request completes, a server-held output when
// the caller releases it.  A worker thread admits queued requests in arrival
// order whenever a slot is idle and the arena can hold the head request,
// enqueues trace -> (validation) -> reuse on the slot's stream through the
// per-view entry points, and polls the slots' completion events.  Requests
// that can never fit the budget are refused at submission.  Latency runs from
// arrival to the worker observing completion.
//
// With `mock` set no HIP call is made: a request "runs" for a modelled time,
// which lets the scheduling logic be tested without a device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "api_internal.hpp"

using namespace ocr;

namespace {

double clock_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// First-fit allocator over [0, size) with coalescing of free neighbours.
class Arena {
   public:
    explicit Arena(size_t size) : size_(size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t &off) {
        bytes = align256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                const size_t rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    bool fits(size_t bytes) const {
        bytes = align256(bytes);
        for (auto &f : free_)
            if (f.second >= bytes) return true;
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align256(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
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
    size_t used() const { return used_; }
    size_t size() const { return size_; }

   private:
    size_t size_, used_ = 0;
    std::map<size_t, size_t> free_;
};

struct Scene {
    const ocr_bvh *bvh;
    std::vector<ocr_gbuffer> views;
};

struct Job {
    uint64_t ticket = 0;
    ocr_request req{};
    int32_t w = 0, h = 0;
    double arrival_ms = 0.0;
    size_t state_bytes = 0;  // records + workspace
    size_t ws_bytes = 0;
    size_t out_bytes = 0;    // server-held output (0 when the caller gave one)
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    Job job;
    size_t state_off = 0, out_off = 0;
    double start_ms = 0.0, mock_end_ms = 0.0;
};

}  // namespace

struct ocr_server {
    ocr_server_options opt{};
    int device = 0;
    char *arena_mem = nullptr;
    Arena *arena = nullptr;
    std::vector<Slot> slots;
    std::deque<Job> queue;
    std::deque<ocr_result> results;
    std::map<uint64_t, std::pair<size_t, size_t>> held;  // ticket -> (offset, bytes) of server-held outputs
    std::vector<double> latencies;
    std::vector<Scene> scenes;
    std::mutex mu;
    std::condition_variable cv;
    std::thread worker;
    bool stop = false;
    uint64_t next_ticket = 1;
    int64_t submitted = 0, completed = 0, failed = 0, refused = 0, waited_for_memory = 0, max_in_flight = 0;
    int64_t admissions = 0;
    size_t peak_used = 0;
    double first_arrival_ms = -1.0, last_done_ms = 0.0;
};

namespace {

bool any_busy(const ocr_server *s) {
    for (const Slot &sl : s->slots)
        if (sl.busy) return true;
    return false;
}

// Enqueue one request's device work on its slot's stream.
ocr_status launch_job(ocr_server *s, Slot &sl) {
    const Job &j = sl.job;
    const ocr_request &r = j.req;
    const Scene &sc = s->scenes[r.scene_id];
    const ocr_gbuffer &gb = sc.views[r.view];
    const size_t px = (size_t)j.w * j.h;
    char *st = s->arena_mem + sl.state_off;
    ocr_occluders occ{(float *)st, (float *)(st + align256(12 * px)), (uint32_t *)(st + 2 * align256(12 * px))};
    void *ws = j.ws_bytes ? (void *)(st + 2 * align256(12 * px) + align256(4 * px)) : nullptr;
    float *out = r.out ? r.out : (float *)(s->arena_mem + sl.out_off);
    ocr_reuse_params p = r.params;
    // the light effects all reuse shadow records
    const int32_t tmode = r.mode == OCR_AO ? OCR_AO : OCR_SHADOW;
    ocr_status rc =
        ocr_trace_occluders(sc.bvh, &gb, tmode, r.ao_radius, &r.light, r.seed, r.sample, &occ, sl.stream);
    if (rc) return rc;
    switch (r.mode) {
        case OCR_AO: rc = ocr_reuse_ao(sc.bvh, &gb, &occ, r.ao_radius, &p, ws, j.ws_bytes, out, sl.stream); break;
        case OCR_SHADOW:
            rc = ocr_reuse_shadow(sc.bvh, &gb, &occ, &r.light, &p, ws, j.ws_bytes, out, sl.stream);
            break;
        case OCR_SHADOW_SOLID_ANGLE:
            rc = ocr_reuse_shadow_solid_angle(sc.bvh, &gb, &occ, &r.light, &p, ws, j.ws_bytes, out, sl.stream);
            break;
        default:
            rc = ocr_reuse_direct_illumination(sc.bvh, &gb, &occ, &r.light, r.radiance, r.albedo, &p, ws, j.ws_bytes,
                                               out, sl.stream);
            break;
    }
    if (rc) return rc;
    return hipEventRecord(sl.done, sl.stream) == hipSuccess ? OCR_OK : OCR_ERR_HIP;
}

void finish(ocr_server *s, Slot &sl, double end_ms, ocr_status st) {
    const Job &j = sl.job;
    ocr_result res{};
    res.ticket = j.ticket;
    res.status = st;
    res.width = j.w;
    res.height = j.h;
    res.out = j.req.out ? j.req.out : (float *)(s->arena_mem + sl.out_off);
    res.arrival_ms = j.arrival_ms;
    res.start_ms = sl.start_ms;
    res.end_ms = end_ms;
    res.latency_ms = end_ms - j.arrival_ms;
    s->arena->release(sl.state_off, j.state_bytes);
    if (j.out_bytes) {
        if (st == OCR_OK) s->held[j.ticket] = {sl.out_off, j.out_bytes};
        else s->arena->release(sl.out_off, j.out_bytes);
    }
    s->results.push_back(res);
    if (st == OCR_OK) s->latencies.push_back(res.latency_ms);
    else s->failed++;
    s->completed++;
    s->last_done_ms = std::max(s->last_done_ms, end_ms);
    sl.busy = false;
}

void worker_loop(ocr_server *s) {
    // (a worker that cannot select the device completes every request with OCR_ERR_HIP)
    const hipError_t dev_e = s->opt.mock ? hipSuccess : hipSetDevice(s->device);
    const int poll_us = s->opt.poll_us > 0 ? s->opt.poll_us : 20;
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        const double t = clock_ms();
        for (Slot &sl : s->slots) {
            if (!sl.busy) continue;
            if (s->opt.mock) {
                if (t >= sl.mock_end_ms) finish(s, sl, sl.mock_end_ms, OCR_OK);
            } else {
                const hipError_t q = hipEventQuery(sl.done);
                if (q == hipSuccess) finish(s, sl, t, OCR_OK);
                else if (q != hipErrorNotReady) finish(s, sl, t, OCR_ERR_HIP);
            }
        }
        // admit in arrival order while a slot is idle and the head fits
        while (!s->queue.empty()) {
            Slot *idle = nullptr;
            for (Slot &sl : s->slots)
                if (!sl.busy) {
                    idle = &sl;
                    break;
                }
            if (!idle) break;
            Job &head = s->queue.front();
            size_t so = 0, oo = 0;
            if (!s->arena->alloc(head.state_bytes, so)) {
                s->waited_for_memory++;
                break;
            }
            if (head.out_bytes && !s->arena->alloc(head.out_bytes, oo)) {
                s->arena->release(so, head.state_bytes);
                s->waited_for_memory++;
                break;
            }
            idle->job = head;
            idle->state_off = so;
            idle->out_off = oo;
            idle->busy = true;
            idle->start_ms = clock_ms();
            s->queue.pop_front();
            s->peak_used = std::max(s->peak_used, s->arena->used());
            int64_t inflight = 0;
            for (Slot &sl : s->slots) inflight += sl.busy;
            s->max_in_flight = std::max(s->max_in_flight, inflight);
            if (s->opt.fault_every > 0 && ++s->admissions % s->opt.fault_every == 0) {
                finish(s, *idle, clock_ms(), OCR_ERR_OOM);  // injected fault
            } else if (s->opt.mock) {
                idle->mock_end_ms = idle->start_ms + s->opt.mock_ns_per_pixel * 1e-6 * idle->job.w * idle->job.h;
            } else {
                const ocr_status rc = dev_e == hipSuccess ? launch_job(s, *idle) : OCR_ERR_HIP;
                if (rc) finish(s, *idle, clock_ms(), rc);
            }
        }
        const bool busy = any_busy(s);
        if (s->stop && s->queue.empty() && !busy) break;
        if (!busy && s->queue.empty()) {
            s->cv.wait(lk);
        } else {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(poll_us));
            lk.lock();
        }
    }
}

void destroy_server(ocr_server *s) {
    for (Slot &sl : s->slots) {
        if (sl.stream) {
            // (teardown: nothing is left to report an error to)
            (void)hipStreamSynchronize(sl.stream);
            (void)hipStreamDestroy(sl.stream);
        }
        if (sl.done) (void)hipEventDestroy(sl.done);
    }
    if (s->arena_mem) (void)hipFree(s->arena_mem);
    delete s->arena;
    delete s;
}

}  // namespace

extern "C" {

double ocr_server_now_ms(void) { return clock_ms(); }

ocr_status ocr_server_create(const ocr_server_options *opt, ocr_server **out) {
    if (!opt || !out) return fail(OCR_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (opt->hbm_budget_bytes < 4096) return fail(OCR_ERR_INVALID_ARG, "budget %zu < 4096 bytes", opt->hbm_budget_bytes);
    if (opt->max_slots < 1 || opt->max_slots > 64) return fail(OCR_ERR_INVALID_ARG, "slots %d not in 1..64", opt->max_slots);
    if (opt->max_queue < 0 || opt->poll_us < 0) return fail(OCR_ERR_INVALID_ARG, "negative queue limit or poll interval");
    if (opt->mock && !(opt->mock_ns_per_pixel >= 0.0)) return fail(OCR_ERR_INVALID_ARG, "bad mock service time");
    if (opt->fault_every < 0) return fail(OCR_ERR_INVALID_ARG, "negative fault_every");
    ocr_server *s = new (std::nothrow) ocr_server;
    if (!s) return fail(OCR_ERR_OOM, "server allocation failed");
    s->opt = *opt;
    s->arena = new Arena(opt->hbm_budget_bytes);
    s->slots.resize(opt->max_slots);
    if (!opt->mock) {
        hipError_t e = hipGetDevice(&s->device);
        if (e == hipSuccess) e = hipMalloc(&s->arena_mem, opt->hbm_budget_bytes);
        if (e != hipSuccess) {
            destroy_server(s);
            return e == hipErrorOutOfMemory ? fail(OCR_ERR_OOM, "arena of %zu bytes", opt->hbm_budget_bytes)
                                            : hip_fail(e, "arena allocation");
        }
        for (Slot &sl : s->slots) {
            e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
            if (e != hipSuccess) {
                destroy_server(s);
                return hip_fail(e, "slot stream");
            }
        }
    }
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return OCR_OK;
}

ocr_status ocr_server_add_scene(ocr_server *s, const ocr_bvh *bvh, const ocr_gbuffer *views, int32_t nviews,
                                int32_t *scene_id) {
    if (!s || !views || nviews < 1 || !scene_id) return fail(OCR_ERR_INVALID_ARG, "bad scene arguments");
    if (!s->opt.mock && !bvh) return fail(OCR_ERR_INVALID_ARG, "bvh is NULL");
    for (int32_t v = 0; v < nviews; ++v) {
        if (s->opt.mock) {
            if (views[v].width < 1 || views[v].height < 1)
                return fail(OCR_ERR_INVALID_ARG, "view %d size %dx%d", v, views[v].width, views[v].height);
        } else if (ocr_status st = check_gbuf(&views[v])) {
            return fail(st, "view %d: %s", v, ocr_last_error());
        }
    }
    std::lock_guard<std::mutex> g(s->mu);
    s->scenes.push_back(Scene{bvh, std::vector<ocr_gbuffer>(views, views + nviews)});
    *scene_id = (int32_t)s->scenes.size() - 1;
    return OCR_OK;
}

ocr_status ocr_server_submit(ocr_server *s, const ocr_request *r, uint64_t *ticket) {
    if (!s || !r || !ticket) return fail(OCR_ERR_INVALID_ARG, "NULL argument");
    const double t = clock_ms();
    if (ocr_status st = check_params(&r->params)) return st;
    if (r->params.accumulate || r->params.validated)
        return fail(OCR_ERR_INVALID_ARG, "accumulate and validated must be 0 in a request");
    LightF L;
    if (r->mode == OCR_AO) {
        if (ocr_status st = check_effect(r->mode, r->ao_radius, &r->light, L)) return st;
    } else if (r->mode >= OCR_SHADOW && r->mode <= OCR_DIRECT_ILLUMINATION) {
        // any emitter density: the per-view entry points take it
        if (ocr_status st = make_light(&r->light, L)) return st;
        if (r->mode == OCR_DIRECT_ILLUMINATION &&
            !(std::isfinite(r->radiance) && r->radiance >= 0.0f && std::isfinite(r->albedo) && r->albedo >= 0.0f))
            return fail(OCR_ERR_INVALID_ARG, "radiance %g and albedo %g must be finite and >= 0",
                        (double)r->radiance, (double)r->albedo);
    } else {
        return fail(OCR_ERR_INVALID_ARG, "request mode %d out of range", r->mode);
    }
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return fail(OCR_ERR_BUSY, "server is stopping");
    if (r->scene_id < 0 || r->scene_id >= (int32_t)s->scenes.size())
        return fail(OCR_ERR_INVALID_ARG, "unknown scene %d", r->scene_id);
    const Scene &sc = s->scenes[r->scene_id];
    if (r->view < 0 || r->view >= (int32_t)sc.views.size())
        return fail(OCR_ERR_INVALID_ARG, "scene %d has no view %d", r->scene_id, r->view);
    Job j;
    j.req = *r;
    j.w = sc.views[r->view].width;
    j.h = sc.views[r->view].height;
    const size_t px = (size_t)j.w * j.h;
    j.ws_bytes = ocr_workspace_bytes(j.w, j.h, &r->params);
    j.state_bytes = 2 * align256(12 * px) + align256(4 * px) + align256(j.ws_bytes);
    j.out_bytes = r->out ? 0 : align256(4 * px);
    const size_t need = j.state_bytes + j.out_bytes;
    if (need > s->arena->size()) {
        s->refused++;
        return fail(OCR_ERR_BUDGET, "request needs %zu bytes, the budget is %zu", need, s->arena->size());
    }
    if (s->opt.max_queue > 0 && (int64_t)s->queue.size() >= s->opt.max_queue)
        return fail(OCR_ERR_BUSY, "queue full (%d)", s->opt.max_queue);
    j.ticket = s->next_ticket++;
    j.arrival_ms = r->arrival_ms > 0.0 ? r->arrival_ms : t;
    if (s->first_arrival_ms < 0.0 || j.arrival_ms < s->first_arrival_ms) s->first_arrival_ms = j.arrival_ms;
    s->queue.push_back(j);
    s->submitted++;
    *ticket = j.ticket;
    s->cv.notify_one();
    return OCR_OK;
}

ocr_status ocr_server_poll(ocr_server *s, ocr_result *out, int32_t max, int32_t *n) {
    if (!s || !n || max < 0 || (max > 0 && !out)) return fail(OCR_ERR_INVALID_ARG, "bad poll arguments");
    std::lock_guard<std::mutex> g(s->mu);
    int32_t k = 0;
    while (k < max && !s->results.empty()) {
        out[k++] = s->results.front();
        s->results.pop_front();
    }
    *n = k;
    return OCR_OK;
}

ocr_status ocr_server_release(ocr_server *s, uint64_t ticket) {
    if (!s) return fail(OCR_ERR_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->held.find(ticket);
    if (it == s->held.end())
        return fail(OCR_ERR_INVALID_ARG, "ticket %llu holds no output", (unsigned long long)ticket);
    s->arena->release(it->second.first, it->second.second);
    s->held.erase(it);
    s->cv.notify_one();
    return OCR_OK;
}

ocr_status ocr_server_drain(ocr_server *s) {
    if (!s) return fail(OCR_ERR_INVALID_ARG, "server is NULL");
    while (true) {
        {
            std::lock_guard<std::mutex> g(s->mu);
            const bool busy = any_busy(s);
            if (s->queue.empty() && !busy) return OCR_OK;
            // nothing in flight and the head does not fit: only releasing
            // server-held outputs can make room
            if (!busy && !s->arena->fits(s->queue.front().state_bytes + s->queue.front().out_bytes) &&
                !s->held.empty())
                return fail(OCR_ERR_BUSY, "queued requests wait for server-held outputs to be released");
        }
        std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
}

ocr_status ocr_server_get_stats(ocr_server *s, ocr_server_stats *st) {
    if (!s || !st) return fail(OCR_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    std::memset(st, 0, sizeof *st);
    st->submitted = s->submitted;
    st->completed = s->completed;
    st->refused = s->refused;
    st->queued = (int64_t)s->queue.size();
    for (const Slot &sl : s->slots) st->in_flight += sl.busy;
    st->waited_for_memory = s->waited_for_memory;
    st->peak_bytes = (int64_t)s->peak_used;
    st->budget_bytes = (int64_t)s->arena->size();
    st->max_in_flight = s->max_in_flight;
    st->failed = s->failed;
    std::vector<double> l = s->latencies;
    if (!l.empty()) {
        std::sort(l.begin(), l.end());
        // nearest-rank percentiles
        auto pct = [&](double q) {
            const size_t k = (size_t)std::ceil(q * (double)l.size());
            return l[std::min(l.size() - 1, k > 0 ? k - 1 : 0)];
        };
        st->p50_ms = pct(0.50);
        st->p99_ms = pct(0.99);
        st->max_ms = l.back();
        double sum = 0.0;
        for (double v : l) sum += v;
        st->mean_ms = sum / (double)l.size();
    }
    if (s->completed > 0 && s->last_done_ms > s->first_arrival_ms)
        st->frames_per_s = (double)s->completed / ((s->last_done_ms - s->first_arrival_ms) * 1e-3);
    return OCR_OK;
}

ocr_status ocr_server_destroy(ocr_server *s) {
    if (!s) return OCR_OK;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        // server-held outputs die with the server; their room lets any
        // request still queued run to completion
        for (auto &h : s->held) s->arena->release(h.second.first, h.second.second);
        s->held.clear();
        s->cv.notify_one();
    }
    if (s->worker.joinable()) s->worker.join();
    destroy_server(s);
    return OCR_OK;
}

}  // extern "C"
