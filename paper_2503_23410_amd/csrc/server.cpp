// Serving loop: per-headset frame requests carrying their gaze arrive at any
// time; a dispatcher thread admits them against an HBM budget, batches every
// admitted request into the next device launch as soon as a launch slot is
// free (continuous batching: late requests join the next launch while
// earlier launches still run), overlaps launches on several streams, and
// reports completion with timestamps for latency statistics.
//
// Scenes, BVHs and layouts stay resident (the headsets reference them); the
// per-request LP buffers and display images come from recycled buffer sets
// whose total size is bounded by the budget.
//
// Requests may carry a completion deadline (a VR frame is useless once its
// display refresh has passed).  The dispatcher keeps a model of device time
// -- a cost per launch plus a cost per request of each headset, corrected
// after each launch by its measured duration -- and the predicted time at
// which the device drains the work already launched.  A launch only takes
// requests that the model says will finish in time; a request that cannot
// finish in time even alone is dropped before it costs device time.  The
// plan also keeps a margin: the worst amount by which a launch recently
// ended after its modelled end, decaying launch by launch, so that a spell of
// slower launches (a hotter device, a host delay) makes the next plans more
// conservative instead of making every request in it late.
//
// A watchdog watches the device's progress, not the age of launches: with
// several launches queued the oldest may legitimately wait long, but some
// launch must complete every watchdog_ms.  When none does, the launched work
// is given up and reported, and the server stops taking work.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "vafr_internal.h"

namespace vafr {
namespace {

using Clock = std::chrono::steady_clock;

struct BufSet {
    float* lp[2] = {nullptr, nullptr};
    float* img[2] = {nullptr, nullptr};
    size_t bytes = 0;
    int64_t key = 0;   // (n_texels, pixels) class
};

struct Pending {
    vafr_request req;
    double submit_ms;
    double due_ms = INFINITY;   // completion deadline on the server clock
    BufSet* bufs = nullptr;
    bool deferred = false;
};

struct Launch {
    std::vector<Pending> reqs;
    hipEvent_t start = nullptr, done = nullptr;
    int stream = 0;
    double launch_ms = 0;
    double pred_ms = 0;       // modelled device time of this launch
    double pred_end_ms = 0;   // modelled completion on the server clock
    double sim_done_ms = 0;   // simulated executor: completion time
    double sim_cost_ms = 0;   // simulated executor: device time of the launch
};

}  // namespace
}  // namespace vafr

struct vafr_server_s {
    vafr_server_config cfg{};
    int device = -1;
    std::chrono::steady_clock::time_point t0;
    std::vector<vafr_headset> headsets;
    std::vector<hipStream_t> streams;
    std::vector<vafr_batch> batches;          // one per stream
    std::vector<hipEvent_t> free_events;
    // buffer pool
    std::multimap<int64_t, vafr::BufSet*> free_sets;
    std::vector<vafr::BufSet*> all_sets;
    std::map<int32_t, vafr::BufSet*> leased;  // result slot -> buffers held by the caller
    size_t bytes_in_use = 0;                  // allocated sets (free or not)
    int32_t next_slot = 1;
    // queues
    std::deque<vafr::Pending> waiting;        // submitted, not yet launched
    std::vector<vafr::Launch> inflight;
    std::deque<vafr_result> done;
    // stats
    int64_t n_submitted = 0, n_completed = 0, n_refused = 0, n_deferred = 0, n_dropped = 0, n_launches = 0;
    int64_t views_launched = 0, n_late = 0, n_superseded = 0, n_stalled = 0;
    // device-time model: launch cost + per-request cost of each headset
    double est_launch_ms = 0;
    std::vector<double> est_req_ms;
    double pred_free_ms = 0;                  // modelled end of the launched work
    double late_margin_ms = 0;                // decaying worst lateness of a launch against its model
    // watchdog
    double progress_ms = 0;                   // last completion, or launch onto an idle device
    bool stalled = false;
    std::vector<vafr::Launch> abandoned;      // launches given up; their buffers stay out of the pool
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    int error = VAFR_OK;
    char error_msg[256] = "";
    std::thread worker;
    double sim_busy_until = 0;                // simulated executor: device timeline
};

namespace vafr {
namespace {

// Decay of the lateness margin per completed launch (it halves over about
// 140 launches, a fraction of a second under load).
constexpr double kMarginDecay = 0.995;

// Launches are planned to end by this fraction of a request's budget: the
// rest absorbs the spread of device times around the model and the delay
// before the dispatcher sees a launch finish.  Under the path-traced
// 8-headset load at 11.1 ms, 0.9 let the slowest served frame overshoot the
// budget by up to 0.24 ms (of about 6,000); 0.85 kept every frame within
// it for 1% fewer frames served.
constexpr double kPlanFraction = 0.85;

double now_ms(vafr_server s) { return std::chrono::duration<double, std::milli>(Clock::now() - s->t0).count(); }

size_t set_bytes(const vafr_headset& h) {
    const vafr_layout L = h.layout;
    return 2 * (size_t)L->n_texels * 16 + 2 * (size_t)L->disp.width * L->disp.height * 16;
}

int64_t set_key(const vafr_headset& h) {
    return h.layout->n_texels * ((int64_t)1 << 32) + (int64_t)h.layout->disp.width * h.layout->disp.height;
}

void free_set(BufSet* b) {
    for (int e = 0; e < 2; ++e) {
        (void)hipFree(b->lp[e]);
        (void)hipFree(b->img[e]);
    }
    delete b;
}

// A buffer set for headset h within the budget, or nullptr (caller holds mu).
BufSet* acquire_set(vafr_server s, const vafr_headset& h) {
    const int64_t key = set_key(h);
    auto it = s->free_sets.find(key);
    if (it != s->free_sets.end()) {
        BufSet* b = it->second;
        s->free_sets.erase(it);
        return b;
    }
    const size_t need = set_bytes(h);
    // evict free sets of other shapes while that makes room
    while (s->bytes_in_use + need > (size_t)s->cfg.hbm_budget_bytes && !s->free_sets.empty()) {
        auto victim = s->free_sets.begin();
        BufSet* v = victim->second;
        s->free_sets.erase(victim);
        s->bytes_in_use -= v->bytes;
        s->all_sets.erase(std::find(s->all_sets.begin(), s->all_sets.end(), v));
        if (s->cfg.simulate) delete v;
        else free_set(v);
    }
    if (s->bytes_in_use + need > (size_t)s->cfg.hbm_budget_bytes) return nullptr;
    BufSet* b = new (std::nothrow) BufSet;
    if (!b) return nullptr;
    b->bytes = need;
    b->key = key;
    bool ok = true;
    for (int e = 0; e < 2 && ok && !s->cfg.simulate; ++e) {
        ok = hipMalloc(&b->lp[e], (size_t)h.layout->n_texels * 16) == hipSuccess &&
             hipMalloc(&b->img[e], (size_t)h.layout->disp.width * h.layout->disp.height * 16) == hipSuccess;
    }
    if (!ok) {
        free_set(b);
        return nullptr;
    }
    s->bytes_in_use += need;
    s->all_sets.push_back(b);
    return b;
}

void release_set(vafr_server s, BufSet* b) { s->free_sets.emplace(b->key, b); }

// Finish a request with an error status and no result slot (caller holds mu).
void push_error(vafr_server s, const Pending& p, int status, double launch_ms, double t) {
    vafr_result r;
    std::memset(&r, 0, sizeof(r));
    r.user_tag = p.req.user_tag;
    r.headset = p.req.headset;
    r.frame = p.req.frame;
    r.status = status;
    r.submit_ms = p.submit_ms;
    r.launch_ms = launch_ms;
    r.done_ms = t;
    s->done.push_back(r);
    ++s->n_dropped;
    s->cv.notify_all();
}

// Finish a request that is not launched with an error status (caller holds
// mu); its buffers go back to the pool.
void finish_dropped(vafr_server s, Pending& p, int status, double t) {
    push_error(s, p, status, t, t);
    if (p.bufs) release_set(s, p.bufs);
    p.bufs = nullptr;
}

// Initial device-time estimate of one request of headset h: rays traced for
// both eyes' LP buffers and pixels written by both reconstructions, at rates
// of the order the device sustains; corrected by measurement after launches.
double initial_request_ms(const vafr_server_config& c, const vafr_headset& h) {
    const double texels = 2.0 * (double)h.layout->n_texels;
    const double pixels = 2.0 * (double)h.layout->disp.width * h.layout->disp.height;
    if (c.simulate) return c.sim_ms_per_mray * texels * 1e-6 + c.sim_ms_per_mpix * pixels * 1e-6;
    const double shadow = h.shading.shadow_rays ? 2.0 : 1.0;
    const double rays_per_texel =
        h.shading.mode == VAFR_SHADE_PATH ? shadow * (1.0 + (double)h.shading.bounces) : shadow;
    return texels * rays_per_texel * 0.25e-6 + pixels * 0.004e-6;
}

void set_error(vafr_server s, int code, const char* msg) {
    if (s->error == VAFR_OK) {
        s->error = code;
        std::snprintf(s->error_msg, sizeof(s->error_msg), "%s", msg);
    }
}

// Launch one batched frame of the admitted requests at the queue head on
// stream k (caller holds mu).
void launch(vafr_server s, int k) {
    Launch L;
    L.stream = k;
    const int max_req = std::max(1, s->cfg.max_views_per_launch / 2);
    const double t_now = now_ms(s);
    const double free_at = std::max(t_now, s->pred_free_ms);
    const double m = s->late_margin_ms;            // deadline checks only; the model's end stays unbiased
    double cost = s->est_launch_ms, due = INFINITY;
    while (!s->waiting.empty() && (int)L.reqs.size() < max_req) {
        Pending& p = s->waiting.front();
        if (!p.bufs) break;                         // head not admitted yet: keep order
        const double c = s->est_req_ms[p.req.headset];
        if (free_at + m + cost + c > std::min(due, p.due_ms)) {
            // Too late in this launch.  If it cannot finish in time in a
            // launch of its own right after this one either, drop it now.
            const double alone = (L.reqs.empty() ? free_at : free_at + cost) + m + s->est_launch_ms + c;
            if (alone > p.due_ms) {
                ++s->n_late;
                finish_dropped(s, p, VAFR_E_LATE, t_now);
                s->waiting.pop_front();
                continue;
            }
            break;
        }
        cost += c;
        due = std::min(due, p.due_ms);
        L.reqs.push_back(p);
        s->waiting.pop_front();
    }
    if (L.reqs.empty()) return;
    L.pred_ms = cost;
    L.pred_end_ms = free_at + cost;
    std::vector<vafr_view> views;
    views.reserve(2 * L.reqs.size());
    for (const Pending& p : L.reqs) {
        const vafr_headset& h = s->headsets[p.req.headset];
        for (int e = 0; e < 2; ++e) {
            vafr_view v;
            std::memset(&v, 0, sizeof(v));
            v.kind = VAFR_VIEW_VAFR;
            v.scene = h.scene;
            v.layout = h.layout;
            v.camera = h.camera[e];
            v.gaze = p.req.gaze;
            v.shading = h.shading;
            v.shading.frame = p.req.frame;
            v.shading.view = (uint32_t)(2 * p.req.headset + e);
            v.lp_rgba_dev = p.bufs->lp[e];
            v.img_rgba_dev = p.bufs->img[e];
            views.push_back(v);
        }
    }
    L.launch_ms = now_ms(s);
    if (s->cfg.simulate) {
        // cost model: fixed launch cost + rays (LP texels) + display pixels
        double mray = 0, mpix = 0;
        for (const Pending& p : L.reqs) {
            const vafr_layout lay = s->headsets[p.req.headset].layout;
            mray += 2e-6 * (double)lay->n_texels;
            mpix += 2e-6 * (double)lay->disp.width * lay->disp.height;
        }
        const double start = std::max(L.launch_ms, s->sim_busy_until);
        L.sim_cost_ms = s->cfg.sim_ms_per_launch + s->cfg.sim_ms_per_mray * mray + s->cfg.sim_ms_per_mpix * mpix;
        L.sim_done_ms = start + L.sim_cost_ms;
        s->sim_busy_until = L.sim_done_ms;
        s->pred_free_ms = L.pred_end_ms;
        if (s->inflight.empty()) s->progress_ms = L.launch_ms;
        ++s->n_launches;
        s->views_launched += (int64_t)views.size();
        s->inflight.push_back(std::move(L));
        return;
    }
    L.start = s->free_events.back();
    s->free_events.pop_back();
    int rc = hipEventRecord(L.start, s->streams[k]) == hipSuccess ? VAFR_OK : VAFR_E_HIP;
    if (rc == VAFR_OK) rc = vafr_batch_run(s->batches[k], views.data(), (int32_t)views.size(), s->streams[k]);
    if (rc == VAFR_OK) {
        L.done = s->free_events.back();
        s->free_events.pop_back();
        if (hipEventRecord(L.done, s->streams[k]) != hipSuccess) rc = VAFR_E_HIP;
    }
    if (rc != VAFR_OK) {
        set_error(s, rc, vafr_last_error());
        for (Pending& p : L.reqs) {
            push_error(s, p, rc, L.launch_ms, L.launch_ms);
            release_set(s, p.bufs);
        }
        if (L.done) s->free_events.push_back(L.done);
        s->free_events.push_back(L.start);
        return;
    }
    s->pred_free_ms = L.pred_end_ms;
    if (s->inflight.empty()) s->progress_ms = L.launch_ms;
    ++s->n_launches;
    s->views_launched += (int64_t)views.size();
    s->inflight.push_back(std::move(L));
}

// The device made no progress for watchdog_ms: give up every launch in
// flight (its buffers stay leased to the abandoned launch, since the device
// may still write them) and every waiting request, and stop taking work
// (caller holds mu).
void abandon(vafr_server s, double t) {
    char msg[160];
    std::snprintf(msg, sizeof(msg), "device made no progress for %.1f ms with %d launch(es) in flight",
                  t - s->progress_ms, (int)s->inflight.size());
    set_error(s, VAFR_E_TIMEOUT, msg);
    s->stalled = true;
    for (Launch& L : s->inflight) {
        for (const Pending& p : L.reqs) {
            push_error(s, p, VAFR_E_TIMEOUT, L.launch_ms, t);
            ++s->n_stalled;
        }
        s->abandoned.push_back(std::move(L));
    }
    s->inflight.clear();
    for (Pending& p : s->waiting) {
        finish_dropped(s, p, VAFR_E_TIMEOUT, t);
        ++s->n_stalled;
    }
    s->waiting.clear();
}

// After launch L finished at time t: correct the model by the ratio of
// measured to modelled device time, and move the modelled end of the work
// still in flight by the error.
void learn(vafr_server s, const Launch& L, double t) {
    double dur = L.pred_ms;
    if (s->cfg.simulate) {
        dur = L.sim_cost_ms;
    } else {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, L.start, L.done) == hipSuccess && ms > 0.0f) dur = ms;
    }
    if (L.pred_ms > 0.0 && dur > 0.0) {
        const double ratio = std::min(4.0, std::max(0.25, dur / L.pred_ms));
        const double f = 0.7 + 0.3 * ratio;
        s->est_launch_ms *= f;
        for (const Pending& p : L.reqs) s->est_req_ms[p.req.headset] *= f;
    }
    const double shift = t - L.pred_end_ms;
    s->late_margin_ms = std::max(shift, s->late_margin_ms * kMarginDecay);
    for (Launch& o : s->inflight) o.pred_end_ms += shift;
    s->pred_free_ms += shift;
    if (s->inflight.size() <= 1) s->pred_free_ms = t;   // only L was in flight: the device is idle
}

void worker_main(vafr_server s) {
    if (!s->cfg.simulate) (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lock(s->mu);
    while (true) {
        // completions
        for (size_t i = 0; i < s->inflight.size();) {
            Launch& L = s->inflight[i];
            const hipError_t q = s->cfg.simulate ? (now_ms(s) >= L.sim_done_ms ? hipSuccess : hipErrorNotReady)
                                                 : hipEventQuery(L.done);
            if (q == hipErrorNotReady) { ++i; continue; }
            const double t = now_ms(s);
            for (Pending& p : L.reqs) {
                vafr_result r;
                std::memset(&r, 0, sizeof(r));
                r.user_tag = p.req.user_tag;
                r.headset = p.req.headset;
                r.frame = p.req.frame;
                r.status = q == hipSuccess ? VAFR_OK : VAFR_E_HIP;
                r.submit_ms = p.submit_ms;
                r.launch_ms = L.launch_ms;
                r.done_ms = t;
                r.slot = s->next_slot++;
                for (int e = 0; e < 2; ++e) {
                    r.img_rgba_dev[e] = p.bufs->img[e];
                    r.lp_rgba_dev[e] = p.bufs->lp[e];
                }
                s->leased[r.slot] = p.bufs;
                s->done.push_back(r);
                ++s->n_completed;
            }
            if (q != hipSuccess) set_error(s, VAFR_E_HIP, "a launched frame failed");
            s->progress_ms = t;
            learn(s, L, t);
            if (L.done) s->free_events.push_back(L.done);
            if (L.start) s->free_events.push_back(L.start);
            s->inflight.erase(s->inflight.begin() + i);
            s->cv.notify_all();
        }
        // watchdog
        const double t = now_ms(s);
        if (s->cfg.watchdog_ms > 0.0 && !s->inflight.empty() && t - s->progress_ms > s->cfg.watchdog_ms)
            abandon(s, t);
        // admission: give buffers to waiting requests in arrival order;
        // drop requests whose deadline already passed
        for (auto it = s->waiting.begin(); it != s->waiting.end();) {
            if (t + s->late_margin_ms + s->est_launch_ms + s->est_req_ms[it->req.headset] > it->due_ms) {
                ++s->n_late;
                finish_dropped(s, *it, VAFR_E_LATE, t);
                it = s->waiting.erase(it);
                continue;
            }
            if (!it->bufs) {
                it->bufs = acquire_set(s, s->headsets[it->req.headset]);
                if (!it->bufs) {                              // wait for memory, keep order
                    if (s->stop) {                            // draining: no memory will come back
                        finish_dropped(s, *it, VAFR_E_BUDGET, t);
                        it = s->waiting.erase(it);
                        continue;
                    }
                    if (!it->deferred) { it->deferred = true; ++s->n_deferred; }
                    break;
                }
            }
            ++it;
        }
        // continuous batching: every free launch slot takes what is ready
        while ((int)s->inflight.size() < s->cfg.max_inflight && !s->waiting.empty() && s->waiting.front().bufs) {
            std::vector<int> busy(std::max<size_t>(1, s->streams.size()), 0);
            for (auto& L : s->inflight) busy[L.stream]++;
            const int k = (int)(std::min_element(busy.begin(), busy.end()) - busy.begin());
            launch(s, k);
        }
        if (s->stop && s->waiting.empty() && s->inflight.empty()) break;
        if (s->inflight.empty() && (s->waiting.empty() || !s->waiting.front().bufs) && !s->stop) {
            s->cv.wait_for(lock, std::chrono::milliseconds(2));
        } else {
            lock.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(50));
            lock.lock();
        }
    }
}

}  // namespace
}  // namespace vafr

using namespace vafr;

extern "C" int vafr_server_create(const vafr_server_config* cfg, vafr_server* out) {
    if (!out || !cfg) return fail(VAFR_E_ARG, "NULL argument");
    *out = nullptr;
    if (cfg->max_views_per_launch < 2 || cfg->max_views_per_launch > 256)
        return fail(VAFR_E_ARG, "max_views_per_launch must be in [2, 256]");
    if (cfg->max_inflight < 1 || cfg->max_inflight > 64) return fail(VAFR_E_ARG, "max_inflight must be in [1, 64]");
    if (cfg->n_streams < 1 || cfg->n_streams > 8) return fail(VAFR_E_ARG, "n_streams must be in [1, 8]");
    if (cfg->hbm_budget_bytes <= 0) return fail(VAFR_E_ARG, "hbm_budget_bytes must be positive");
    if (cfg->max_queue < 1) return fail(VAFR_E_ARG, "max_queue must be positive");
    if (cfg->simulate != 0 && cfg->simulate != 1) return fail(VAFR_E_ARG, "simulate must be 0 or 1");
    if (cfg->simulate && (!(cfg->sim_ms_per_launch >= 0) || !(cfg->sim_ms_per_mray >= 0) || !(cfg->sim_ms_per_mpix >= 0)))
        return fail(VAFR_E_ARG, "simulated costs must be >= 0");
    if (!(cfg->frame_budget_ms >= 0) || !std::isfinite(cfg->frame_budget_ms))
        return fail(VAFR_E_ARG, "frame_budget_ms must be finite and >= 0");
    if (cfg->latest_only != 0 && cfg->latest_only != 1) return fail(VAFR_E_ARG, "latest_only must be 0 or 1");
    if (!(cfg->watchdog_ms >= 0) || !std::isfinite(cfg->watchdog_ms))
        return fail(VAFR_E_ARG, "watchdog_ms must be finite and >= 0");
    int n_dev = 0;
    if (!cfg->simulate && (hipGetDeviceCount(&n_dev) != hipSuccess || n_dev == 0))
        return fail(VAFR_E_HIP, "no HIP device available");
    vafr_server s = new (std::nothrow) vafr_server_s;
    if (!s) return fail(VAFR_E_OOM, "server allocation failed");
    s->cfg = *cfg;
    s->t0 = Clock::now();
    s->est_launch_ms = cfg->simulate ? cfg->sim_ms_per_launch : 0.03;
    auto bail = [&](int code) {
        vafr_server_destroy(s);
        return code;
    };
    if (!cfg->simulate && hipGetDevice(&s->device) != hipSuccess) return bail(fail(VAFR_E_HIP, "hipGetDevice failed"));
    for (int k = 0; k < cfg->n_streams && !cfg->simulate; ++k) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
            return bail(fail(VAFR_E_HIP, "stream creation failed"));
        s->streams.push_back(st);
        vafr_batch b;
        if (int rc = vafr_batch_create(cfg->max_views_per_launch, &cfg->batch, &b)) return bail(rc);
        s->batches.push_back(b);
    }
    // two timing events (start, done) per launch in flight, plus spares
    for (int k = 0; k < 2 * (cfg->max_inflight + 1) && !cfg->simulate; ++k) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return bail(fail(VAFR_E_HIP, "event creation failed"));
        s->free_events.push_back(e);
    }
    s->worker = std::thread(worker_main, s);
    *out = s;
    return VAFR_OK;
}

extern "C" int vafr_server_add_headset(vafr_server s, const vafr_headset* h, int32_t* id) {
    if (!s || !h || !id) return fail(VAFR_E_ARG, "NULL argument");
    if (!h->layout || (!h->scene && !s->cfg.simulate)) return fail(VAFR_E_ARG, "headset needs a scene and a layout");
    if (h->layout->kind != VAFR_LAYOUT_VAFR) return fail(VAFR_E_ARG, "headset layouts must be VaFR layouts");
    for (int e = 0; e < 2; ++e)
        if (int rc = check_camera(&h->camera[e])) return rc;
    if (int rc = check_shading(&h->shading)) return rc;
    std::lock_guard<std::mutex> lock(s->mu);
    if (set_bytes(*h) > (size_t)s->cfg.hbm_budget_bytes)
        return fail(VAFR_E_BUDGET, "one frame of this headset does not fit the HBM budget");
    s->headsets.push_back(*h);
    s->est_req_ms.push_back(initial_request_ms(s->cfg, *h));
    *id = (int32_t)s->headsets.size() - 1;
    return VAFR_OK;
}

extern "C" int vafr_server_submit(vafr_server s, const vafr_request* r) {
    if (!s || !r) return fail(VAFR_E_ARG, "NULL argument");
    if (int rc = check_gaze(r->gaze)) return rc;
    std::lock_guard<std::mutex> lock(s->mu);
    if (s->stop) return fail(VAFR_E_ARG, "server is draining");
    if (s->stalled) return fail(VAFR_E_TIMEOUT, "server stopped after a device stall: %s", s->error_msg);
    if (r->headset < 0 || r->headset >= (int32_t)s->headsets.size()) return fail(VAFR_E_ARG, "unknown headset");
    ++s->n_submitted;
    if ((int64_t)s->waiting.size() >= s->cfg.max_queue) {
        ++s->n_refused;
        return fail(VAFR_E_BUDGET, "request queue is full (%d waiting)", (int)s->waiting.size());
    }
    Pending p;
    p.req = *r;
    p.submit_ms = now_ms(s);
    double budget = s->cfg.frame_budget_ms > 0.0 ? s->cfg.frame_budget_ms : INFINITY;
    if (r->deadline_ms > 0.0) budget = std::min(budget, r->deadline_ms);
    p.due_ms = p.submit_ms + kPlanFraction * budget;
    if (s->cfg.latest_only) {
        for (auto it = s->waiting.begin(); it != s->waiting.end();) {
            if (it->req.headset != r->headset) { ++it; continue; }
            ++s->n_superseded;
            finish_dropped(s, *it, VAFR_E_LATE, p.submit_ms);
            it = s->waiting.erase(it);
        }
    }
    s->waiting.push_back(p);
    s->cv.notify_all();
    return VAFR_OK;
}

extern "C" int vafr_server_poll(vafr_server s, vafr_result* out, int32_t max, int32_t* n_out) {
    if (!s || !n_out || (max > 0 && !out)) return fail(VAFR_E_ARG, "NULL argument");
    std::lock_guard<std::mutex> lock(s->mu);
    int32_t n = 0;
    while (n < max && !s->done.empty()) {
        out[n++] = s->done.front();
        s->done.pop_front();
    }
    *n_out = n;
    if (n == 0 && s->error != VAFR_OK) return fail(s->error, "%s", s->error_msg);
    return VAFR_OK;
}

extern "C" int vafr_server_release(vafr_server s, int32_t slot) {
    if (!s) return fail(VAFR_E_ARG, "server is NULL");
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->leased.find(slot);
    if (it == s->leased.end()) return fail(VAFR_E_ARG, "unknown result slot %d", slot);
    release_set(s, it->second);
    s->leased.erase(it);
    s->cv.notify_all();
    return VAFR_OK;
}

extern "C" int vafr_server_wait_idle(vafr_server s, int32_t timeout_ms) {
    if (!s) return fail(VAFR_E_ARG, "server is NULL");
    std::unique_lock<std::mutex> lock(s->mu);
    const bool idle = s->cv.wait_for(lock, std::chrono::milliseconds(timeout_ms < 0 ? 0 : timeout_ms),
                                     [&] { return s->waiting.empty() && s->inflight.empty(); });
    return idle ? VAFR_OK : fail(VAFR_E_BUDGET, "server still busy after %d ms", timeout_ms);
}

extern "C" int vafr_server_get_stats(vafr_server s, vafr_server_stats* out) {
    if (!s || !out) return fail(VAFR_E_ARG, "NULL argument");
    std::lock_guard<std::mutex> lock(s->mu);
    out->submitted = s->n_submitted;
    out->completed = s->n_completed;
    out->refused = s->n_refused;
    out->deferred = s->n_deferred;
    out->dropped = s->n_dropped;
    out->launches = s->n_launches;
    out->views_launched = s->views_launched;
    out->bytes_in_use = (int64_t)s->bytes_in_use;
    out->waiting = (int32_t)s->waiting.size();
    out->inflight = (int32_t)s->inflight.size();
    out->late = s->n_late;
    out->superseded = s->n_superseded;
    out->stalled = s->n_stalled;
    return VAFR_OK;
}

extern "C" void vafr_server_destroy(vafr_server s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    bool hung = false;
    for (auto& L : s->abandoned) hung = hung || (!s->cfg.simulate && hipEventQuery(L.done) == hipErrorNotReady);
    if (hung) {
        // Abandoned work is still on the device: waiting for it may never
        // end and freeing what it uses is unsafe, so every device object
        // (streams, events, batches, buffers) is leaked.
        for (auto b : s->all_sets) delete b;
        delete s;
        return;
    }
    for (auto& L : s->abandoned) {
        if (L.done) (void)hipEventDestroy(L.done);
        if (L.start) (void)hipEventDestroy(L.start);
    }
    for (auto b : s->batches) vafr_batch_destroy(b);
    for (auto st : s->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    for (auto e : s->free_events) (void)hipEventDestroy(e);
    for (auto& L : s->inflight) {
        if (L.done) (void)hipEventDestroy(L.done);
        if (L.start) (void)hipEventDestroy(L.start);
    }
    for (auto b : s->all_sets) {
        if (s->cfg.simulate) delete b;
        else free_set(b);
    }
    delete s;
}
