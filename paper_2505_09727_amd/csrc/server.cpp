// Continuous-batching request server (esp_server_* in esp.h).
//
// A scheduler thread owns one HIP stream and one device arena sized by the
// HBM budget. Every iteration it admits waiting requests in arrival order
// while their state fits in the arena (and below the active-request limit),
// rebuilds the launch set when the active set changed, evaluates one step of
// every active request with one launch per pipeline phase, applies the
// per-step drift to the resident positions, and retires requests that have
// done all their steps (freeing their memory for the next admissions).
//
// Iterations overlap: iteration k is enqueued (with the copy of its energies
// into one of two pinned result tables and an event) before the scheduler
// waits for iteration k - 1, so admission, launch-set assembly and result
// handling on the host run while the device computes. A request leaves the
// active set when its last step is enqueued; its memory and output slot are
// released when that step's results arrive.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "assembly.hpp"
#include "esp.h"
#include "kernels.hpp"
#include "plan.hpp"

using namespace esp;

namespace {

thread_local std::string s_err;

esp_status sfail(esp_status s, const std::string& m) {
    s_err = m;
    return s;
}

// First-fit allocator of byte ranges in [0, capacity), 256-byte aligned.
class Arena {
  public:
    explicit Arena(size_t cap) : cap_(cap) { free_[0] = cap; }
    // offset or SIZE_MAX
    size_t alloc(size_t bytes) {
        bytes = (bytes + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first, rem = it->second - bytes;
                free_.erase(it);
                if (rem) free_[off + bytes] = rem;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                sizes_[off] = bytes;
                return off;
            }
        }
        return SIZE_MAX;
    }
    void release(size_t off) {
        auto s = sizes_.find(off);
        if (s == sizes_.end()) return;
        size_t bytes = s->second;
        sizes_.erase(s);
        used_ -= bytes;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t capacity() const { return cap_; }

  private:
    size_t cap_, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
    std::map<size_t, size_t> sizes_;
};

double now_s(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct ServerRequest {
    uint64_t id = 0;
    int tile = 0;
    esp_request req{};
    std::vector<float> pos, q;          // host copies (freed on admission)
    esp_params prm{};
    size_t bytes = 0;
    size_t arena_off = SIZE_MAX;
    int out_slot = -1;
    SystemSlot slot;
    int steps_done = 0;       // steps whose results arrived
    int steps_launched = 0;   // steps enqueued
    esp_result res{};
    std::vector<float> phi_out, F_out;  // kept outputs of the last step
};

struct esp_server {
    esp_server_opts opts{};
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    int device = 0;
    hipStream_t stream = nullptr;
    unsigned char* arena_base = nullptr;
    std::unique_ptr<Arena> arena;
    double* d_out = nullptr;            // max_active x kOutDoubles
    double* h_out[2] = {nullptr, nullptr};  // pinned copies, one per iteration in flight
    hipEvent_t ev[2] = {nullptr, nullptr};  // completion of the iteration using table k & 1
    std::vector<int> free_out;
    TableStore tables;
    std::mutex tables_mu;
    LaunchSet ls;
    // shared state
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::unique_ptr<ServerRequest>> to_plan;    // submitted, parameters not yet resolved
    std::map<uint64_t, std::unique_ptr<ServerRequest>> planned;  // planned ahead of an earlier request
    uint64_t next_release = 1;                              // next id to hand to the scheduler
    std::deque<std::unique_ptr<ServerRequest>> arrivals;   // planned, not yet seen by the scheduler
    std::deque<std::unique_ptr<ServerRequest>> waiting;    // seen, waiting for memory
    std::vector<std::unique_ptr<ServerRequest>> active;    // scheduler-owned, steps still to enqueue
    std::vector<std::unique_ptr<ServerRequest>> finishing; // last step enqueued, results pending
    std::deque<esp_result> done;
    std::unordered_map<uint64_t, std::unique_ptr<ServerRequest>> kept;  // finished, outputs kept
    std::vector<double> latencies;
    uint64_t next_id = 1;
    int64_t submitted = 0, admitted = 0, completed = 0, failed = 0, iterations = 0;
    double particle_steps = 0.0, busy_s = 0.0, t_first_submit = -1.0, t_last_done = 0.0;
    double build_s = 0.0, admit_s = 0.0, step_s = 0.0;
    bool stop = false;
    std::string fatal;
    std::thread worker;
    std::vector<std::thread> planners;
    int planning_n = 0;      // requests held by planner threads
    std::condition_variable cv_plan;

    void loop();
    void plan_loop();
    // One enqueued iteration: the requests it stepped and when.
    struct Inflight {
        int64_t k;
        double t_launch;
        std::vector<ServerRequest*> reqs;
    };
    std::deque<Inflight> inflight;
    // Wait for the oldest enqueued iteration and take its results (caller
    // does not hold mu). False after a device error (fatal is set).
    bool complete_oldest();
    bool admit_locked(ServerRequest* r);
    void retire(ServerRequest* r);
};

namespace {

size_t request_bytes(const esp_params& p, int64_t N) {
    const size_t io = ((12 * N + 255) & ~size_t(255)) + 3 * ((4 * N + 255) & ~size_t(255)) +
                      ((12 * N + 255) & ~size_t(255));  // pos, q, phi, F (FP32)
    return io + scratch_bytes(p, N);
}

}  // namespace

// Place a waiting request in the arena (caller holds mu). False when it does
// not fit now.
bool esp_server::admit_locked(ServerRequest* r) {
    if ((int)active.size() >= opts.max_active || free_out.empty()) return false;
    const size_t off = arena->alloc(r->bytes);
    if (off == SIZE_MAX) return false;
    r->arena_off = off;
    r->out_slot = free_out.back();
    free_out.pop_back();
    unsigned char* base = arena_base + off;
    const size_t N = (size_t)r->req.N;
    auto a = [](size_t x) { return (x + 255) & ~size_t(255); };
    float* pos = reinterpret_cast<float*>(base);
    float* q = reinterpret_cast<float*>(base + a(12 * N));
    float* phi = reinterpret_cast<float*>(base + a(12 * N) + a(4 * N));
    float* F = reinterpret_cast<float*>(base + a(12 * N) + 2 * a(4 * N));
    unsigned char* scr = base + a(12 * N) + 3 * a(4 * N) + a(12 * N);
    r->slot.prm = r->prm;
    r->slot.N = r->req.N;
    r->slot.scr = carve_scratch(scr, r->prm, r->req.N);
    r->slot.scr.out = d_out + (size_t)kOutDoubles * r->out_slot;
    r->slot.pos = pos;
    r->slot.q = q;
    r->slot.phi = phi;
    r->slot.F = F;
    r->slot.seed = r->req.seed;
    r->slot.drift = (float)r->req.drift;
    // pageable copies are staged synchronously, so the host vectors can go
    (void)hipMemcpyAsync(pos, r->pos.data(), 12 * N, hipMemcpyHostToDevice, stream);
    (void)hipMemcpyAsync(q, r->q.data(), 4 * N, hipMemcpyHostToDevice, stream);
    std::vector<float>().swap(r->pos);
    std::vector<float>().swap(r->q);
    r->res.t_admit = now_s(t0);
    ++admitted;
    return true;
}

void esp_server::retire(ServerRequest* r) {
    if (opts.keep_outputs) {
        const size_t N = (size_t)r->req.N;
        r->phi_out.resize(N);
        r->F_out.resize(3 * N);
        (void)hipMemcpy(r->phi_out.data(), r->slot.phi, 4 * N, hipMemcpyDeviceToHost);
        (void)hipMemcpy(r->F_out.data(), r->slot.F, 12 * N, hipMemcpyDeviceToHost);
    }
    arena->release(r->arena_off);
    free_out.push_back(r->out_slot);
}

// Parameter resolution and table classes off the submission path: the first
// request of a (grid, tolerance) class costs ~0.1 s of host work.
void esp_server::plan_loop() {
    (void)hipSetDevice(device);
    for (;;) {
        std::unique_ptr<ServerRequest> r;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_plan.wait(lk, [&] { return stop || !to_plan.empty(); });
            if (stop) return;
            r = std::move(to_plan.front());
            to_plan.pop_front();
            ++planning_n;
        }
        std::string msg;
        esp_params req{};
        req.precision = 32;
        esp_status st = resolve_params(r->req.L, r->req.N, r->req.tol, &req, &r->prm, msg);
        if (st == ESP_OK) {
            r->prm.tile = r->tile;
            const DeviceClass* cls = nullptr;
            std::lock_guard<std::mutex> tl(tables_mu);
            st = tables.get(r->prm, &cls, msg);
            r->slot.cls = cls;
        }
        std::lock_guard<std::mutex> lk(mu);
        --planning_n;
        const uint64_t id = r->id;
        if (st != ESP_OK) {
            r->res.status = st;
            r->res.t_done = now_s(t0);
            ++failed;
            done.push_back(r->res);
            cv_done.notify_all();
            r.reset();  // a hole in the release order
        } else {
            r->res.nf = r->prm.nf;
            r->res.P = r->prm.P;
        }
        // planners finish out of order; the scheduler sees submission order
        planned.emplace(id, std::move(r));
        bool any = false;
        for (auto it = planned.begin(); it != planned.end() && it->first == next_release;
             it = planned.erase(it), ++next_release)
            if (it->second) {
                arrivals.push_back(std::move(it->second));
                any = true;
            }
        if (any) cv_work.notify_one();
    }
}

bool esp_server::complete_oldest() {
    Inflight it = std::move(inflight.front());
    inflight.pop_front();
    const hipError_t e = hipEventSynchronize(ev[it.k & 1]);
    const double t_end = now_s(t0);
    std::lock_guard<std::mutex> lk(mu);
    if (e != hipSuccess) {
        fatal = std::string("device error: ") + hipGetErrorString(e);
        stop = true;
        cv_done.notify_all();
        return false;
    }
    step_s += t_end - it.t_launch;
    const double* table = h_out[it.k & 1];
    for (ServerRequest* r : it.reqs) {
        const double* o = table + (size_t)kOutDoubles * r->out_slot;
        if (r->steps_done == 0) r->res.E_first = o[0];
        r->res.E_last = o[0];
        ++r->steps_done;
        if (r->steps_done == 1 && std::fabs(o[1]) > 1e-6 * o[2]) r->res.status = ESP_E_NOT_NEUTRAL;
        if (r->steps_done < r->req.nsteps) continue;
        // the last step's results: release the request
        retire(r);
        r->res.t_done = t_end;
        ++completed;
        particle_steps += (double)r->req.N * r->req.nsteps;
        latencies.push_back(r->res.t_done - r->res.t_submit);
        t_last_done = t_end;
        done.push_back(r->res);
        auto f = std::find_if(finishing.begin(), finishing.end(), [&](const auto& p) { return p.get() == r; });
        if (opts.keep_outputs) kept[r->id] = std::move(*f);
        finishing.erase(f);
    }
    busy_s += now_s(t0) - t_end;  // host time on the results (not the wait)
    cv_done.notify_all();
    return true;
}

void esp_server::loop() {
    (void)hipSetDevice(device);
    bool changed = false;
    int64_t k = 0;  // iterations enqueued
    for (;;) {
        bool launch = false;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] {
                return stop || !arrivals.empty() || !waiting.empty() || !active.empty() || !inflight.empty();
            });
            if (stop) return;
            while (!arrivals.empty()) {
                waiting.push_back(std::move(arrivals.front()));
                arrivals.pop_front();
            }
            const double ta = now_s(t0);
            while (!waiting.empty() && admit_locked(waiting.front().get())) {
                active.push_back(std::move(waiting.front()));
                waiting.pop_front();
                changed = true;
            }
            admit_s += now_s(t0) - ta;
            if (active.empty() && inflight.empty() && finishing.empty() && !waiting.empty()) {
                // nothing fits although nothing runs: the head request can never be admitted
                auto r = std::move(waiting.front());
                waiting.pop_front();
                r->res.status = ESP_E_BUSY;
                r->res.t_done = now_s(t0);
                ++failed;
                done.push_back(r->res);
                cv_done.notify_all();
                continue;
            }
            launch = !active.empty();
        }
        if (launch) {
            const double t_iter = now_s(t0);
            std::string msg;
            if (changed) {
                const double tb = now_s(t0);
                std::vector<SystemSlot> slots;
                slots.reserve(active.size());
                for (auto& r : active) slots.push_back(r->slot);
                // one stream: no pipeline lanes (one spread and one gather
                // launch per window width)
                if (ls.build(slots, 32, stream, msg, 1) != ESP_OK) {
                    std::lock_guard<std::mutex> lk(mu);
                    fatal = msg;
                    stop = true;
                    cv_done.notify_all();
                    return;
                }
                changed = false;
                build_s += now_s(t0) - tb;
            }
            const Launch& L = ls.launch();
            // one step of every active request
            hipError_t e = hipSuccess;
            for (int ph = 0; ph < 3 && e == hipSuccess; ++ph) e = launch_prepare(L, ph);
            if (e == hipSuccess) e = launch_local(L);
            for (const Group& G : ls.groups())
                if (e == hipSuccess) e = launch_spread(L, G);
            for (int pass = 0; pass < 3; ++pass)
                for (const FftGroup& G : ls.fft_groups())
                    if (e == hipSuccess) e = launch_fft(L, G, pass, 0);
            for (const Group& G : ls.groups())
                if (e == hipSuccess) e = launch_gather(L, G);
            if (e == hipSuccess) e = launch_finalize(L, nullptr);
            // drift for the next step of requests that continue
            bool any_drift = false;
            for (size_t s = 0; s < active.size(); ++s) {
                ServerRequest* r = active[s].get();
                const int step =
                    (r->steps_launched + 1 < r->req.nsteps && r->req.drift > 0) ? r->steps_launched + 1 : 0;
                ls.set_step((int)s, step);
                any_drift |= step > 0;
            }
            if (e == hipSuccess && any_drift) {
                if (ls.upload_descriptors(msg) != ESP_OK) e = hipErrorUnknown;
                if (e == hipSuccess) e = launch_drift(L);
            }
            if (e == hipSuccess)
                e = hipMemcpyAsync(h_out[k & 1], d_out, sizeof(double) * kOutDoubles * opts.max_active,
                                   hipMemcpyDeviceToHost, stream);
            if (e == hipSuccess) e = hipEventRecord(ev[k & 1], stream);
            if (e != hipSuccess) {
                std::lock_guard<std::mutex> lk(mu);
                fatal = std::string("device error: ") + hipGetErrorString(e);
                stop = true;
                cv_done.notify_all();
                return;
            }
            Inflight it{k, t_iter, {}};
            it.reqs.reserve(active.size());
            {
                std::lock_guard<std::mutex> lk(mu);
                std::vector<std::unique_ptr<ServerRequest>> still;
                for (auto& rp : active) {
                    it.reqs.push_back(rp.get());
                    if (++rp->steps_launched >= rp->req.nsteps) {
                        finishing.push_back(std::move(rp));
                        changed = true;
                    } else {
                        still.push_back(std::move(rp));
                    }
                }
                active.swap(still);
                ++iterations;
                busy_s += now_s(t0) - t_iter;
            }
            inflight.push_back(std::move(it));
            ++k;
        }
        // take the results of the previous iteration while this one runs (or
        // of the last one when nothing new was enqueued)
        if (launch) {
            while (inflight.size() > 1)
                if (!complete_oldest()) return;
        } else if (!inflight.empty()) {
            if (!complete_oldest()) return;
        }
    }
}

extern "C" {

const char* esp_server_last_error(void) { return s_err.c_str(); }

esp_status esp_server_create(const esp_server_opts* opts, esp_server** out) {
    if (!out) return sfail(ESP_E_INVALID, "out is NULL");
    *out = nullptr;
    std::unique_ptr<esp_server> s(new (std::nothrow) esp_server());
    if (!s) return sfail(ESP_E_NOMEM, "host allocation failed");
    if (opts) s->opts = *opts;
    if (s->opts.hbm_budget_bytes == 0) s->opts.hbm_budget_bytes = (size_t)16 << 30;
    if (s->opts.max_active <= 0) s->opts.max_active = 4096;
    if (hipGetDevice(&s->device) != hipSuccess) return sfail(ESP_E_DEVICE, "no device");
    if (hipStreamCreate(&s->stream) != hipSuccess) return sfail(ESP_E_DEVICE, "hipStreamCreate failed");
    if (hipMalloc(&s->arena_base, s->opts.hbm_budget_bytes) != hipSuccess) {
        (void)hipStreamDestroy(s->stream);
        return sfail(ESP_E_NOMEM, "cannot allocate the HBM budget");
    }
    s->arena.reset(new Arena(s->opts.hbm_budget_bytes));
    for (int b = 0; b < 2; ++b)
        if (hipHostMalloc((void**)&s->h_out[b], sizeof(double) * kOutDoubles * s->opts.max_active,
                          hipHostMallocDefault) != hipSuccess ||
            hipEventCreateWithFlags(&s->ev[b], hipEventDisableTiming) != hipSuccess)
            return sfail(ESP_E_NOMEM, "cannot allocate the result tables");
    if (hipMalloc(&s->d_out, sizeof(double) * kOutDoubles * s->opts.max_active) != hipSuccess)
        return sfail(ESP_E_NOMEM, "cannot allocate the result table");
    (void)hipMemset(s->d_out, 0, sizeof(double) * kOutDoubles * s->opts.max_active);
    for (int i = s->opts.max_active - 1; i >= 0; --i) s->free_out.push_back(i);
    esp_server* raw = s.get();
    raw->worker = std::thread([raw] { raw->loop(); });
    for (int t = 0; t < 4; ++t) raw->planners.emplace_back([raw] { raw->plan_loop(); });
    *out = s.release();
    return ESP_OK;
}

esp_status esp_server_submit(esp_server* s, const esp_request* rq, uint64_t* id) {
    if (!s || !rq || !rq->pos || !rq->q) return sfail(ESP_E_INVALID, "NULL argument");
    if (rq->N < 2 || rq->nsteps < 1) return sfail(ESP_E_INVALID, "need N >= 2 and nsteps >= 1");
    if (!(rq->L > 0) || !(rq->tol >= 1e-8 && rq->tol <= 1e-2)) return sfail(ESP_E_INVALID, "bad box or tolerance");
    auto r = std::make_unique<ServerRequest>();
    r->req = *rq;
    // shape of the default parameters (cheap); the rest is resolved by the planner
    esp_params shape{};
    shape.precision = 32;
    shape.nf = grid_size(rq->L, 1.25);
    shape.P = order_for_tol(rq->tol);
    if (shape.nf > 144) return sfail(ESP_E_UNSUPPORTED, "box needs a grid above 144 points per side");
    r->tile = choose_tile(shape.nf, 0, std::min<long long>(512, std::max<long long>(8, rq->N / 512)));
    shape.tile = r->tile;
    r->bytes = request_bytes(shape, rq->N);
    if (r->bytes > s->opts.hbm_budget_bytes) return sfail(ESP_E_BUSY, "request larger than the HBM budget");
    r->pos.assign(rq->pos, rq->pos + 3 * rq->N);
    r->q.assign(rq->q, rq->q + rq->N);
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->fatal.empty()) return sfail(ESP_E_DEVICE, s->fatal);
    r->id = s->next_id++;
    r->res.id = r->id;
    r->res.tag = rq->tag;
    r->res.status = ESP_OK;
    r->res.nsteps = rq->nsteps;
    r->res.N = rq->N;
    r->res.nf = shape.nf;
    r->res.P = shape.P;
    r->res.t_submit = now_s(s->t0);
    if (s->t_first_submit < 0) s->t_first_submit = r->res.t_submit;
    if (id) *id = r->id;
    ++s->submitted;
    s->to_plan.push_back(std::move(r));
    s->cv_plan.notify_one();
    return ESP_OK;
}

esp_status esp_server_poll(esp_server* s, esp_result* out, int max, int* n) {
    if (!s || !n || (max > 0 && !out)) return sfail(ESP_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    int k = 0;
    while (k < max && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    *n = k;
    if (!s->fatal.empty()) return sfail(ESP_E_DEVICE, s->fatal);
    return ESP_OK;
}

esp_status esp_server_fetch(esp_server* s, uint64_t id, float* phi, float* F) {
    if (!s) return sfail(ESP_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->kept.find(id);
    if (it == s->kept.end()) return sfail(ESP_E_INVALID, "no kept outputs for this id (keep_outputs off, unknown, or fetched)");
    if (phi) std::memcpy(phi, it->second->phi_out.data(), it->second->phi_out.size() * sizeof(float));
    if (F) std::memcpy(F, it->second->F_out.data(), it->second->F_out.size() * sizeof(float));
    s->kept.erase(it);
    return ESP_OK;
}

esp_status esp_server_wait(esp_server* s, double timeout_s) {
    if (!s) return sfail(ESP_E_INVALID, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    const bool ok = s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] {
        return !s->fatal.empty() ||
               (s->to_plan.empty() && s->planned.empty() && s->arrivals.empty() && s->waiting.empty() &&
                s->active.empty() && s->finishing.empty() && s->planning_n == 0);
    });
    if (!s->fatal.empty()) return sfail(ESP_E_DEVICE, s->fatal);
    return ok ? ESP_OK : sfail(ESP_E_BUSY, "timed out with requests still queued or running");
}

esp_status esp_server_get_stats(esp_server* s, esp_server_stats* st) {
    if (!s || !st) return sfail(ESP_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(st, 0, sizeof(*st));
    st->submitted = s->submitted;
    st->admitted = s->admitted;
    st->completed = s->completed;
    st->failed = s->failed;
    st->active = (int64_t)(s->active.size() + s->finishing.size());
    st->waiting = (int64_t)(s->waiting.size() + s->arrivals.size() + s->planned.size() + s->to_plan.size() +
                            s->planning_n);
    st->iterations = s->iterations;
    st->particle_steps = s->particle_steps;
    st->busy_s = s->busy_s;
    st->span_s = s->completed ? s->t_last_done - s->t_first_submit : 0.0;
    st->bytes_in_use = s->arena->used();
    st->bytes_peak = s->arena->peak();
    st->build_s = s->build_s;
    st->admit_s = s->admit_s;
    st->step_s = s->step_s;
    if (!s->latencies.empty()) {
        std::vector<double> v = s->latencies;
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) {
            const double x = p * (v.size() - 1);
            const size_t i = (size_t)x;
            const double f = x - i;
            return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
        };
        st->p50_latency_s = pct(0.50);
        st->p99_latency_s = pct(0.99);
        st->max_latency_s = v.back();
    }
    return ESP_OK;
}

void esp_server_destroy(esp_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    s->cv_plan.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (auto& t : s->planners)
        if (t.joinable()) t.join();
    (void)hipStreamSynchronize(s->stream);
    (void)hipFree(s->arena_base);
    (void)hipFree(s->d_out);
    for (int b = 0; b < 2; ++b) {
        if (s->h_out[b]) (void)hipHostFree(s->h_out[b]);
        if (s->ev[b]) (void)hipEventDestroy(s->ev[b]);
    }
    (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // extern "C"
