// pins_server.cpp -- serving runtime: continuous admission of solve requests
// into running batches.  Each worker thread owns a live batch (pins_live.h) on
// its own HIP stream and device arena.  Between two outer iterations of its
// batch a worker admits queued requests (arrival order, the batch's cost
// family, while a slot and arena room are free); each request runs its own
// K outer iterations and leaves the batch when they are done, so requests that
// arrive while others are on the GPU join them at the next outer-iteration
// boundary, and the batches of different workers overlap on the device.  Each
// instance's arithmetic does not depend on the batch it shares, so a result is
// bitwise the one its problem gets alone.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "pins.h"
#include "pins_live.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    pins_problem prob{};                 // pointers into the owned copies below
    std::vector<double> a, b, C, x, y;   // host copies of the inputs
    std::vector<double> alpha, beta;     // host outputs
    pins_result res{};
    int rc = 0;
    bool done = false;
    Clock::time_point t_submit, t_done;
};

bool grid_family(const pins_problem& p) { return p.kind == PINS_COST_GRID; }

// The solver's marginal rules (positive, finite, sum 1 within 1e-10), checked
// at submission so that an invalid request never fails a whole batch.
bool marginal_ok(const double* v, int len) {
    double s = 0.0;
    for (int i = 0; i < len; ++i) {
        if (!(v[i] > 0.0) || !std::isfinite(v[i])) return false;
        s += v[i];
    }
    return std::fabs(s - 1.0) <= 1e-10;
}

bool all_finite(const double* v, size_t len) {
    for (size_t i = 0; i < len; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

}  // namespace

struct pins_server {
    int device = 0;
    int max_batch = 1;
    size_t budget = 0;
    pins_params params{};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<int64_t> queue;
    std::map<int64_t, std::unique_ptr<Request>> reqs;
    int64_t next = 1;
    bool stop = false;
    std::vector<std::thread> workers;
    std::string err;
};

namespace {

// Default device arena of a worker's live batch when hbm_budget is 0.
constexpr size_t DEFAULT_ARENA = (size_t)4 << 30;

void complete(pins_server* S, Request* r, int rc, const pins_result* res) {
    // caller holds S->mu
    if (res) r->res = *res;
    else std::memset(&r->res, 0, sizeof(r->res));
    r->res.status = rc;
    r->res.alpha = r->alpha.data();
    r->res.beta = r->beta.data();
    r->res.X = nullptr;
    r->rc = rc;
    r->done = true;
    r->t_done = Clock::now();
}

// One worker: a live batch on its own stream.  Between two rounds (outer
// iterations of the batch) it admits queued requests -- arrival order, the
// batch's cost family, while a slot and arena room are free (a request that
// cannot fit even into an empty batch is completed with PINS_ENOMEM) -- then
// runs one round and completes the requests whose K outer iterations are done.
void worker_loop(pins_server* S) {
    if (hipSetDevice(S->device) != hipSuccess) (void)hipGetLastError();
    std::string err;
    pins::LiveBatch* B = pins::live_create(S->device, S->params, S->max_batch,
                                           S->budget > 0 ? S->budget : DEFAULT_ARENA, &err);
    if (!B) {
        std::lock_guard<std::mutex> lk(S->mu);
        S->err = err.empty() ? "worker set-up failed" : err;
    }
    std::vector<pins::LiveDone> done;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty() || pins::live_count(B) > 0; });
            if (S->queue.empty() && pins::live_count(B) == 0) break;  // stopping and nothing left
            for (auto it = S->queue.begin(); it != S->queue.end();) {
                Request* r = S->reqs[*it].get();
                if (!B) {  // no live batch on this worker: its requests fail
                    complete(S, r, PINS_EDEVICE, nullptr);
                    it = S->queue.erase(it);
                    continue;
                }
                if (pins::live_count(B) > 0 && grid_family(r->prob) != pins::live_grid(B)) {
                    ++it;
                    continue;
                }
                if (pins::live_admit(B, *it, r->prob, r->alpha.data(), r->beta.data())) {
                    it = S->queue.erase(it);
                    continue;
                }
                if (pins::live_count(B) == 0) {  // does not fit into an empty batch
                    complete(S, r, PINS_ENOMEM, nullptr);
                    it = S->queue.erase(it);
                    continue;
                }
                break;  // no room now: later requests wait their turn
            }
        }
        S->cv_done.notify_all();
        if (!B) continue;
        done.clear();
        const int rc = pins::live_round(B, done, &err);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            for (const pins::LiveDone& d : done) {
                auto f = S->reqs.find(d.id);
                if (f != S->reqs.end()) complete(S, f->second.get(), d.rc, &d.res);
            }
            if (rc < 0) S->err = err.empty() ? "device error in a live batch" : err;
        }
        S->cv_done.notify_all();
    }
    pins::live_destroy(B);
}

}  // namespace

extern "C" {

int pins_server_create(int device, int workers, int max_batch, size_t hbm_budget, const pins_params* p,
                       pins_server** out) {
    if (!out || !p || workers < 1 || workers > 4 || max_batch < 1) return PINS_EINVAL;
    if (p->shift_mode != PINS_SHIFT_IMPLICIT || p->hvp == 2) return PINS_EUNSUPPORTED;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        (void)hipGetLastError();
        return PINS_EDEVICE;
    }
    // validate the parameters through the planner on a small grid problem
    // (the planner reads no input array)
    const double marg[4] = {0.25, 0.25, 0.25, 0.25};
    pins_problem probe{};
    probe.kind = PINS_COST_GRID;
    probe.m = probe.n = 4;
    probe.grid_s = 2;
    probe.a = marg;
    probe.b = marg;
    size_t ws = 0;
    if (pins_workspace_bytes(&probe, 1, p, &ws) != PINS_OK) return PINS_EINVAL;  // validates the parameters
    auto* S = new pins_server;
    S->device = device;
    S->max_batch = max_batch;
    S->budget = hbm_budget;
    S->params = *p;
    for (int w = 0; w < workers; ++w) S->workers.emplace_back(worker_loop, S);
    *out = S;
    return PINS_OK;
}

int pins_server_submit(pins_server* S, const pins_problem* prob, int64_t* ticket) {
    if (!S || !prob || !ticket || !prob->a || !prob->b || prob->m < 1 || prob->n < 1) return PINS_EINVAL;
    size_t ws = 0;
    if (pins_workspace_bytes(prob, 1, &S->params, &ws) != PINS_OK) return PINS_EINVAL;
    if (prob->kind == PINS_COST_DENSE && !prob->C) return PINS_EINVAL;
    if (prob->kind == PINS_COST_POINTS && (!prob->x || !prob->y || prob->d < 1)) return PINS_EINVAL;
    if (!marginal_ok(prob->a, prob->m) || !marginal_ok(prob->b, prob->n)) return PINS_EINVAL;
    // a non-finite cost would fail the batch it joins: rejected here
    if (prob->kind == PINS_COST_DENSE && !all_finite(prob->C, (size_t)prob->m * prob->n)) return PINS_EINVAL;
    if (prob->kind == PINS_COST_POINTS && (!all_finite(prob->x, (size_t)prob->m * prob->d) ||
                                           !all_finite(prob->y, (size_t)prob->n * prob->d)))
        return PINS_EINVAL;
    auto r = std::make_unique<Request>();
    r->prob = *prob;
    r->a.assign(prob->a, prob->a + prob->m);
    r->b.assign(prob->b, prob->b + prob->n);
    if (prob->kind == PINS_COST_DENSE) r->C.assign(prob->C, prob->C + (size_t)prob->m * prob->n);
    if (prob->kind == PINS_COST_POINTS) {
        r->x.assign(prob->x, prob->x + (size_t)prob->m * prob->d);
        r->y.assign(prob->y, prob->y + (size_t)prob->n * prob->d);
    }
    // the request's problem points at its own copies (read at admission)
    r->prob.a = r->a.data();
    r->prob.b = r->b.data();
    r->prob.C = r->C.empty() ? nullptr : r->C.data();
    r->prob.x = r->x.empty() ? nullptr : r->x.data();
    r->prob.y = r->y.empty() ? nullptr : r->y.data();
    r->alpha.assign(prob->m, 0.0);
    r->beta.assign(prob->n, 0.0);
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) return PINS_EINVAL;
        *ticket = S->next++;
        S->queue.push_back(*ticket);
        S->reqs[*ticket] = std::move(r);
    }
    S->cv_work.notify_one();
    return PINS_OK;
}

int pins_server_wait(pins_server* S, int64_t ticket, pins_result* res, double* latency_ms) {
    if (!S || !res) return PINS_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return PINS_EINVAL;
    Request* r = it->second.get();
    S->cv_done.wait(lk, [&] { return r->done; });
    double* ua = res->alpha;
    double* ub = res->beta;
    *res = r->res;
    res->alpha = ua;
    res->beta = ub;
    res->X = nullptr;
    if (ua) std::memcpy(ua, r->alpha.data(), r->alpha.size() * sizeof(double));
    if (ub) std::memcpy(ub, r->beta.data(), r->beta.size() * sizeof(double));
    if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    const int rc = r->rc;
    S->reqs.erase(it);
    return rc;
}

const char* pins_server_last_error(const pins_server* S) {
    if (!S) return "null server";
    return S->err.c_str();
}

void pins_server_destroy(pins_server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    for (auto& t : S->workers) t.join();
    delete S;
}

}  // extern "C"
