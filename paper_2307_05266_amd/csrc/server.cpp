// Request server: continuous batching of permeability solves on one GPU.
//
// Requests (a geometry, a force, a preconditioner, a tolerance and a
// precision) enter a FIFO queue.  A fixed number of slots, each a host worker
// thread with its own non-blocking HIP stream, take requests from the head of
// the queue as soon as a slot is free and the request's device bytes (bounded
// by stokes_estimate_bytes) fit in what the HBM budget has left; a request
// that arrives while others run is admitted the moment a slot and memory free
// up, and its kernels overlap with theirs on the device.  A slot that takes a
// mixed-precision request also takes the queued requests that can share its
// context (same box size, force, preconditioner and tolerance, as many as
// the member and cell caps and the budget allow, in queue order) and solves
// them as one batched context (stokes_setup_batch): every kernel launch then
// advances all of them, which amortises the per-launch latency that bounds
// small solves.  FP64 requests get a context each (stokes_setup_on_stream).
// Each context allocates in its stream's order, so setting up or tearing down
// one never waits for the others; its Krylov state stays resident for the
// whole solve, and its inner iterations replay captured HIP graphs.  A
// request's arithmetic does not depend on its batch or on the other work on
// the device, so its result is bitwise the same alone or in the mix.
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
    bool valid = true;        // mask bytes are 0 or 1
    bool done = false;
    stokes_request_result res{};
};

}  // namespace

struct stokes_server {
    int device = 0;
    int slots = 1;
    int64_t budget = 0;
    int max_members = 32;             // requests sharing one batched context
    int64_t max_cells = int64_t(1) << 21;   // voxels of one batched context (members x N^3)
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
    int64_t batches = 0, batched_requests = 0;
    bool stop = false;
    std::vector<std::thread> workers;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

void fill_result(stokes_request_result& o, stokes_status st, const stokes_report& rep) {
    o.status = st;
    o.k_hat = rep.k_hat;
    o.outer_iters = rep.outer_iters;
    o.inner_A_iters = rep.inner_A_iters;
    o.inner_S_iters = rep.inner_S_iters;
    o.rel_res = rep.rel_res;
    o.div_norm = rep.div_norm;
}

// One FP64 request on a context of its own.
void run_single(stokes_server* srv, Request* r, hipStream_t stream) {
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
    fill_result(o, st, rep);
    o.t_end = srv->now();
}

// Mixed-precision requests of one size, force, preconditioner and tolerance
// on one batched context.  When the batch cannot be set up as a whole, each
// request runs as a batch of its own, so one request's error stays its own.
void run_batch(stokes_server* srv, const std::vector<Request*>& b, hipStream_t stream) {
    const int B = (int)b.size();
    std::vector<const uint8_t*> masks(B);
    for (int m = 0; m < B; ++m) masks[m] = b[m]->mask.data();
    stokes_ctx* ctx = nullptr;
    stokes_status st = stokes_setup_batch(&ctx, masks.data(), B, b[0]->N, b[0]->force, 0u, stream);
    if (st != STOKES_OK && B > 1) {
        for (Request* r : b) run_batch(srv, std::vector<Request*>{r}, stream);
        return;
    }
    stokes_report rep{};
    stokes_status solved = st;
    if (st == STOKES_OK) solved = stokes_solve(ctx, b[0]->precond, b[0]->tol, &rep);
    int64_t info[12] = {};
    if (ctx && stokes_info(ctx, info) != STOKES_OK) info[9] = 0;
    const double t = srv->now();
    for (int m = 0; m < B; ++m) {
        stokes_request_result& o = b[m]->res;
        stokes_report mr{};
        stokes_status ms = st;
        if (st == STOKES_OK) {
            ms = stokes_batch_result(ctx, m, &mr, nullptr, nullptr);
            if (ms == STOKES_OK) ms = (stokes_status)mr.status;
            else ms = solved;
        }
        fill_result(o, ms, mr);
        o.device_bytes = info[9] / B;
        o.t_end = t;
    }
    if (ctx) stokes_destroy(ctx);
}

bool mask_valid(const Request* r) {
    for (uint8_t v : r->mask)
        if (v > 1) return false;
    return true;
}

bool can_share(const Request* a, const Request* b) {
    return a->precision == 1 && b->precision == 1 && a->N == b->N && a->precond == b->precond &&
           a->tol == b->tol && a->force[0] == b->force[0] && a->force[1] == b->force[1] &&
           a->force[2] == b->force[2] && b->valid;
}

void worker(stokes_server* srv) {
    (void)hipSetDevice(srv->device);
    hipStream_t stream = nullptr;
    const bool have_stream = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess;
    std::vector<Request*> batch;
    for (;;) {
        int64_t charge = 0;
        batch.clear();
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            srv->work_cv.wait(lk, [srv] {
                return srv->stop ||
                       (!srv->queue.empty() && srv->in_use + srv->queue.front()->bytes <= srv->budget);
            });
            if (srv->stop) break;
            Request* head = srv->queue.front();
            srv->queue.pop_front();
            batch.push_back(head);
            charge = head->bytes;
            if (head->precision == 1 && head->valid) {
                const int64_t n3 = (int64_t)head->N * head->N * head->N;
                const int64_t cap = std::min<int64_t>(srv->max_members, std::max<int64_t>(1, srv->max_cells / n3));
                for (auto it = srv->queue.begin(); it != srv->queue.end() && (int64_t)batch.size() < cap;) {
                    Request* r = *it;
                    if (can_share(head, r) && srv->in_use + charge + r->bytes <= srv->budget) {
                        batch.push_back(r);
                        charge += r->bytes;
                        it = srv->queue.erase(it);
                    } else {
                        ++it;
                    }
                }
            }
            const double t = srv->now();
            for (Request* r : batch) {
                r->res.t_start = t;
                r->res.batch_members = (int)batch.size();
            }
            srv->in_use += charge;
            srv->peak = std::max(srv->peak, srv->in_use);
            srv->running += (int)batch.size();
            srv->peak_running = std::max(srv->peak_running, srv->running);
            ++srv->batches;
            srv->batched_requests += (int64_t)batch.size();
        }
        if (!have_stream) {
            for (Request* r : batch) {
                r->res.status = STOKES_E_DEVICE;
                r->res.t_end = srv->now();
            }
        } else if (batch[0]->precision == 1 && batch[0]->valid) {
            run_batch(srv, batch, stream);
        } else {
            run_single(srv, batch[0], stream);
        }
        for (Request* r : batch) {
            r->mask.clear();
            r->mask.shrink_to_fit();
        }
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->in_use -= charge;
            srv->running -= (int)batch.size();
            srv->completed += (int64_t)batch.size();
            for (Request* r : batch) r->done = true;
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
    r->valid = mask_valid(r.get());
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

stokes_status stokes_server_set_batching(stokes_server* srv, int max_members, int64_t max_cells) {
    if (!srv || max_members < 1 || max_members > 32 || max_cells < 1) return STOKES_E_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->max_members = max_members;
    srv->max_cells = max_cells;
    return STOKES_OK;
}

stokes_status stokes_server_stats(stokes_server* srv, int64_t stats[10]) {
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
    stats[8] = srv->batches;
    stats[9] = srv->batched_requests;
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
