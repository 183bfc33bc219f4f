// pins_server.cpp -- serving runtime: continuous admission of solve requests
// onto concurrent batched solves (one worker thread, context and HIP stream
// each).  A worker that becomes free takes every queued request it can (in
// arrival order, same cost-kind family, at most max_batch, workspace within the
// HBM budget, at least one) and solves them in one pins_solve_batch_device
// call; requests that arrive while other batches are on the GPU are admitted
// as workers free up, and the batches of different workers overlap on the
// device.  Each instance's arithmetic does not depend on its batch, so a result
// is bitwise the one its problem gets alone.
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

// Device staging of one batch: inputs and outputs of every request, carved
// from one allocation that grows as needed.
struct Staging {
    void* base = nullptr;
    size_t bytes = 0;
    ~Staging() {
        if (base) (void)hipFree(base);
    }
    bool reserve(size_t need) {
        if (need <= bytes) return true;
        if (base) (void)hipFree(base);
        base = nullptr;
        bytes = 0;
        if (hipMalloc(&base, need) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        bytes = need;
        return true;
    }
};

size_t doubles_of(const pins_problem& p) {
    size_t c = (size_t)2 * (p.m + p.n);  // a, b, alpha, beta
    if (p.kind == PINS_COST_DENSE) c += (size_t)p.m * p.n;
    if (p.kind == PINS_COST_POINTS) c += (size_t)(p.m + p.n) * p.d;
    return c;
}

void worker_loop(pins_server* S) {
    if (hipSetDevice(S->device) != hipSuccess) return;
    pins_ctx* ctx = nullptr;
    const int crc = pins_create(S->device, &ctx);
    hipStream_t st = nullptr;
    // non-blocking: no implicit synchronisation with other workers' work through the null stream
    const bool ok = crc == PINS_OK && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    Staging stage;
    pins_params p = S->params;
    p.streams = 0;  // this worker is one lane
    for (;;) {
        std::vector<Request*> batch;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty(); });
            if (S->queue.empty()) break;  // stopping and nothing left
            // admission: arrival order, one cost-kind family, at most max_batch,
            // workspace within the budget (the first request is always taken)
            const bool fam = grid_family(S->reqs[S->queue.front()]->prob);
            std::vector<pins_problem> probs;
            for (auto it = S->queue.begin(); it != S->queue.end() && (int)batch.size() < S->max_batch;) {
                Request* r = S->reqs[*it].get();
                if (grid_family(r->prob) != fam) {
                    ++it;
                    continue;
                }
                probs.push_back(r->prob);
                size_t ws = 0;
                if (!batch.empty() && S->budget > 0 &&
                    (pins_workspace_bytes(probs.data(), (int)probs.size(), &p, &ws) != PINS_OK || ws > S->budget)) {
                    probs.pop_back();
                    break;
                }
                batch.push_back(r);
                it = S->queue.erase(it);
            }
        }
        const int cnt = (int)batch.size();
        int rc = ok ? PINS_OK : PINS_EDEVICE;
        std::vector<pins_problem> dp(cnt);
        std::vector<pins_result> dr(cnt);
        if (rc == PINS_OK) {
            size_t need = 0;
            for (Request* r : batch) need += doubles_of(r->prob) * sizeof(double) + 256;
            if (!stage.reserve(need)) rc = PINS_ENOMEM;
        }
        if (rc == PINS_OK) {
            char* at = (char*)stage.base;
            auto put = [&](const std::vector<double>& v) {
                double* d = (double*)at;
                if (!v.empty() && hipMemcpyAsync(d, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice,
                                                 st) != hipSuccess)
                    rc = PINS_EDEVICE;
                at += v.size() * sizeof(double);
                return d;
            };
            for (int q = 0; q < cnt; ++q) {
                Request* r = batch[q];
                dp[q] = r->prob;
                dp[q].a = put(r->a);
                dp[q].b = put(r->b);
                dp[q].C = r->C.empty() ? nullptr : put(r->C);
                dp[q].x = r->x.empty() ? nullptr : put(r->x);
                dp[q].y = r->y.empty() ? nullptr : put(r->y);
                std::memset(&dr[q], 0, sizeof(pins_result));
                dr[q].alpha = (double*)at;
                at += (size_t)r->prob.m * sizeof(double);
                dr[q].beta = (double*)at;
                at += (size_t)r->prob.n * sizeof(double);
                at = (char*)(((uintptr_t)at + 255) & ~(uintptr_t)255);
            }
        }
        if (rc == PINS_OK) rc = pins_solve_batch_device(ctx, dp.data(), cnt, &p, dr.data(), st);
        std::string msg = (rc < 0 && ctx) ? pins_last_error(ctx) : "";
        for (int q = 0; q < cnt && rc >= 0; ++q) {
            Request* r = batch[q];
            if (hipMemcpyAsync(r->alpha.data(), dr[q].alpha, r->alpha.size() * sizeof(double), hipMemcpyDeviceToHost,
                               st) != hipSuccess ||
                hipMemcpyAsync(r->beta.data(), dr[q].beta, r->beta.size() * sizeof(double), hipMemcpyDeviceToHost,
                               st) != hipSuccess)
                rc = PINS_EDEVICE;
        }
        if (rc >= 0 && hipStreamSynchronize(st) != hipSuccess) rc = PINS_EDEVICE;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            const auto now = Clock::now();
            for (int q = 0; q < cnt; ++q) {
                Request* r = batch[q];
                r->res = dr[q];
                r->res.alpha = r->alpha.data();
                r->res.beta = r->beta.data();
                r->res.X = nullptr;
                r->rc = rc < 0 ? rc : dr[q].status;
                r->done = true;
                r->t_done = now;
            }
            if (rc < 0) S->err = msg.empty() ? "device error in a served batch" : msg;
        }
        S->cv_done.notify_all();
    }
    if (st) (void)hipStreamDestroy(st);
    if (ctx) pins_destroy(ctx);
}

}  // namespace

extern "C" {

int pins_server_create(int device, int workers, int max_batch, size_t hbm_budget, const pins_params* p,
                       pins_server** out) {
    if (!out || !p || workers < 1 || workers > 4 || max_batch < 1) return PINS_EINVAL;
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
