// Request server: continuous batching of permeability solves on one GPU.
//
// Requests (a geometry, a force, a preconditioner, a tolerance and a
// precision) enter a FIFO queue.  A fixed number of slots, each a host worker
// thread with its own non-blocking HIP stream, take requests from the head of
// the queue as soon as a slot is free and the request's device bytes (bounded
// by stokes_estimate_bytes) fit in what the HBM budget has left; a request
// that arrives while others run is admitted the moment a slot and memory free
// up, and its kernels overlap with theirs on the device (each slot's stream
// maps onto its own hardware queue when enough are configured).  Each request
// gets its own context (stokes_setup_on_stream: stream-ordered allocation, so
// setting up or tearing down one request never waits for the others); its
// Krylov state stays resident in that context for the whole solve, and its
// inner iterations replay captured HIP graphs.  The solve of a request is the
// same sequence of kernels with the same deterministic reductions whether it
// runs alone or among others, so its result is bitwise the same.
//
// Only the public C-ABI of the solver is used here.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/stokes_server.h"

namespace {

struct Request {
    int64_t id = 0;
    int N = 0;
    std::vector<uint8_t> mask;
    double force[3] = {1.0, 0.0, 0.0};
    stokes_precond precond = STOKES_SIMPLE;
    double tol = 1e-8;
    int precision = 0;
    int64_t bytes = 0;        // admission charge
    bool done = false;
    stokes_request_result res{};
};

}  // namespace

struct stokes_server {
    int device = 0;
    int slots = 1;
    int64_t budget = 0;
    std::chrono::steady_clock::time_point t0;

    std::mutex mu;
    std::condition_variable work_cv;   // queue changed / memory freed / stop
    std::condition_variable done_cv;   // a request finished
    std::deque<Request*> queue;
    std::map<int64_t, std::unique_ptr<Request>> all;
    int64_t next_id = 1;
    int64_t in_use = 0, peak = 0;
    int64_t submitted = 0, completed = 0;
    int running = 0, peak_running = 0;
    bool stop = false;
    std::vector<std::thread> workers;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

void run_request(stokes_server* srv, Request* r, hipStream_t stream) {
    stokes_request_result& o = r->res;
    stokes_ctx* ctx = nullptr;
    stokes_status st = stokes_setup_on_stream(&ctx, r->mask.data(), r->N, r->force, 0u, stream);
    if (st == STOKES_OK && r->precision == 1) st = stokes_set_option(ctx, "precision", 1.0);
    stokes_report rep{};
    if (st == STOKES_OK) st = stokes_solve(ctx, r->precond, r->tol, &rep);
    if (ctx) {
        int64_t info[12] = {};
        if (stokes_info(ctx, info) == STOKES_OK) o.device_bytes = info[9];
        stokes_destroy(ctx);
    }
    o.status = st;
    o.k_hat = rep.k_hat;
    o.outer_iters = rep.outer_iters;
    o.inner_A_iters = rep.inner_A_iters;
    o.inner_S_iters = rep.inner_S_iters;
    o.rel_res = rep.rel_res;
    o.div_norm = rep.div_norm;
    o.t_end = srv->now();
    r->mask.clear();
    r->mask.shrink_to_fit();
}

void worker(stokes_server* srv) {
    (void)hipSetDevice(srv->device);
    hipStream_t stream = nullptr;
    const bool have_stream = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess;
    for (;;) {
        Request* r = nullptr;
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            srv->work_cv.wait(lk, [srv] {
                return srv->stop ||
                       (!srv->queue.empty() && srv->in_use + srv->queue.front()->bytes <= srv->budget);
            });
            if (srv->stop) break;
            r = srv->queue.front();
            srv->queue.pop_front();
            r->res.t_start = srv->now();
            srv->in_use += r->bytes;
            srv->peak = std::max(srv->peak, srv->in_use);
            ++srv->running;
            srv->peak_running = std::max(srv->peak_running, srv->running);
        }
        if (have_stream) {
            run_request(srv, r, stream);
        } else {
            r->res.status = STOKES_E_DEVICE;
            r->res.t_end = srv->now();
        }
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->in_use -= r->bytes;
            --srv->running;
            ++srv->completed;
            r->done = true;
        }
        srv->work_cv.notify_all();
        srv->done_cv.notify_all();
    }
    if (have_stream) (void)hipStreamDestroy(stream);
}

}  // namespace

extern "C" {

stokes_status stokes_server_create(stokes_server** out, int slots, int64_t hbm_budget_bytes) {
    if (!out || slots < 1 || slots > 64 || hbm_budget_bytes <= 0) return STOKES_E_ARG;
    stokes_server* srv = new (std::nothrow) stokes_server();
    if (!srv) return STOKES_E_NOMEM;
    if (hipGetDevice(&srv->device) != hipSuccess) {
        delete srv;
        return STOKES_E_DEVICE;
    }
    srv->slots = slots;
    srv->budget = hbm_budget_bytes;
    srv->t0 = std::chrono::steady_clock::now();
    try {
        for (int q = 0; q < slots; ++q) srv->workers.emplace_back(worker, srv);
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->stop = true;
        }
        srv->work_cv.notify_all();
        for (auto& t : srv->workers) t.join();
        delete srv;
        return STOKES_E_NOMEM;
    }
    *out = srv;
    return STOKES_OK;
}

stokes_status stokes_server_submit(stokes_server* srv, const uint8_t* mask, int N, const double force[3],
                                   stokes_precond precond, double tol, int precision, int64_t* id) {
    if (!srv || !mask || !force || !id) return STOKES_E_ARG;
    if (precond != STOKES_UZAWA && precond != STOKES_SIMPLE) return STOKES_E_ARG;
    if (!(tol > 0.0 && tol < 1.0)) return STOKES_E_ARG;
    int64_t bytes = 0;
    const stokes_status est = stokes_estimate_bytes(N, 0u, precision, &bytes);
    if (est != STOKES_OK) return est;
    if (bytes > srv->budget) return STOKES_E_LIMIT;
    auto r = std::unique_ptr<Request>(new (std::nothrow) Request());
    if (!r) return STOKES_E_NOMEM;
    try {
        r->mask.assign(mask, mask + (size_t)N * N * N);
    } catch (const std::bad_alloc&) {
        return STOKES_E_NOMEM;
    }
    r->N = N;
    std::memcpy(r->force, force, sizeof(r->force));
    r->precond = precond;
    r->tol = tol;
    r->precision = precision;
    r->bytes = bytes;
    r->res.N = N;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop) return STOKES_E_STATE;
        r->id = srv->next_id++;
        r->res.id = r->id;
        r->res.t_submit = srv->now();
        *id = r->id;
        srv->queue.push_back(r.get());
        srv->all[r->id] = std::move(r);
        ++srv->submitted;
    }
    srv->work_cv.notify_all();
    return STOKES_OK;
}

stokes_status stokes_server_wait(stokes_server* srv, int64_t id, stokes_request_result* out) {
    if (!srv || !out) return STOKES_E_ARG;
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->all.find(id);
    if (it == srv->all.end()) return STOKES_E_ARG;
    Request* r = it->second.get();
    srv->done_cv.wait(lk, [r] { return r->done; });
    *out = r->res;
    return STOKES_OK;
}

stokes_status stokes_server_stats(stokes_server* srv, int64_t stats[8]) {
    if (!srv || !stats) return STOKES_E_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    stats[0] = srv->submitted;
    stats[1] = srv->completed;
    stats[2] = (int64_t)srv->queue.size();
    stats[3] = srv->running;
    stats[4] = srv->in_use;
    stats[5] = srv->peak;
    stats[6] = srv->peak_running;
    stats[7] = srv->budget;
    return STOKES_OK;
}

double stokes_server_clock(stokes_server* srv) { return srv ? srv->now() : 0.0; }

void stokes_server_destroy(stokes_server* srv) {
    if (!srv) return;
    {
        std::unique_lock<std::mutex> lk(srv->mu);
        // requests still queued are cancelled; running ones finish
        for (Request* r : srv->queue) {
            r->res.status = STOKES_E_STATE;
            r->done = true;
        }
        srv->queue.clear();
        srv->stop = true;
    }
    srv->work_cv.notify_all();
    srv->done_cv.notify_all();
    for (auto& t : srv->workers) t.join();
    delete srv;
}

}  // extern "C"
