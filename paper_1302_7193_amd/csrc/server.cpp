// Serving runtime: continuous batching of independent solves.
//
// pcg_submit queues a request (descriptor, options, host b and x) and
// returns at once.  max_active worker threads, each with its own HIP stream
// and its own cache of problem objects (one per grid shape), admit requests
// in arrival order whenever a worker is idle and the request's device bytes
// (b, x and its solve workspace) fit both the HBM budget and the
// caller-provided device arena.  An admitted request is copied in, solved by
// the fused iteration (HIP-graph chunks, built without stream capture so the
// workers never interfere), copied out and its arena block is
// released, which may admit the next request.  Requests of different shapes
// overlap on the device through the worker streams.  Each request's kernels,
// launch shapes and reduction orders depend only on its own descriptor and
// options, so its result is the same alone and in any mix.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <mutex>
#include <sstream>
#include <string>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "arena.h"
#include "problem.h"

namespace pcg {

size_t request_bytes(const pcg_problem_desc& d, const pcg_solve_opts& o);
pcg_status solve(pcg_problem* P, const double* b, double* x, void* workspace, size_t ws_bytes,
                 const pcg_solve_opts& o, int64_t nrhs, pcg_result* res, hipStream_t s);
std::string validate(const pcg_problem_desc& d);

}  // namespace pcg

extern "C" pcg_status pcg_problem_create(const pcg_problem_desc* desc, pcg_problem** out);
extern "C" void pcg_problem_destroy(pcg_problem* p);
extern "C" void pcg_default_opts(pcg_solve_opts* o);
extern "C" size_t pcg_last_error(char* buf, size_t n);

namespace {

using Clock = std::chrono::steady_clock;

enum class ReqState { Queued, Running, Done, Cancelled };

struct Request {
    uint64_t ticket = 0;
    pcg_problem_desc desc{};
    pcg_solve_opts opts{};
    const double* b_host = nullptr;   // or device pointers when device_io
    double* x_host = nullptr;
    bool device_io = false;
    hipEvent_t ready = nullptr;       // device_io: b and x are ready once this fires
    size_t need = 0;
    size_t offset = 0;
    ReqState state = ReqState::Queued;
    pcg_result result{};
    pcg_status status = PCG_E_AGAIN;
    std::string error;                // worker's message for a failed solve
    Clock::time_point t_submit;
};

using DescKey = std::tuple<int32_t, int32_t, int32_t, double, double, double, double, double,
                           double, int32_t, int32_t>;

DescKey key_of(const pcg_problem_desc& d)
{
    return DescKey(d.nx, d.ny, d.nz, d.dx, d.dy, d.height, d.grading, d.k_h, d.k_v, d.bc_x, d.bc_y);
}

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

struct pcg_server {
    pcg_server_opts opts{};
    int device = 0;
    char* arena_base = nullptr;
    pcg::Arena arena;
    size_t admitted_bytes = 0, peak_bytes = 0;
    int active = 0, peak_active = 0;
    bool stop = false;
    uint64_t next_ticket = 1;
    uint64_t n_submitted = 0, n_completed = 0, n_cancelled = 0, n_rejected = 0;
    std::deque<std::shared_ptr<Request>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> tickets;
    std::mutex mu;
    std::condition_variable cv_admit;   // workers: queue or memory changed
    std::condition_variable cv_done;    // waiters: a request finished
    std::vector<std::thread> workers;

    // Under mu: take the head request if it can be admitted now.
    std::shared_ptr<Request> try_admit()
    {
        if (queue.empty()) return nullptr;
        auto& r = queue.front();
        if (!pcg::admissible(opts.hbm_budget_bytes, admitted_bytes, r->need, active,
                             opts.max_active))
            return nullptr;
        size_t off = 0;
        if (!arena.alloc(r->need, &off)) return nullptr;
        auto req = r;
        queue.pop_front();
        req->offset = off;
        req->state = ReqState::Running;
        admitted_bytes += req->need;
        peak_bytes = std::max(peak_bytes, admitted_bytes);
        ++active;
        peak_active = std::max(peak_active, active);
        return req;
    }

    void worker_main()
    {
        (void)hipSetDevice(device);
        hipStream_t stream = nullptr;
        const bool have_stream = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess;
        std::map<DescKey, pcg_problem*> problems;
        for (;;) {
            std::shared_ptr<Request> req;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_admit.wait(lk, [&] { return stop || (req = try_admit()) != nullptr; });
                if (!req) break;   // stopping and nothing admitted
            }
            pcg_result res{};
            pcg_status st = have_stream ? run(*req, problems, stream, &res) : PCG_E_DEVICE;
            std::string err;
            if (st != PCG_OK && st != PCG_E_NOCONV && st != PCG_E_BREAKDOWN) {
                char buf[512];
                pcg_last_error(buf, sizeof(buf));   // this worker thread's message
                err = have_stream ? buf : "pcg server: could not create a worker stream";
            }
            if (req->ready) {
                (void)hipEventDestroy(req->ready);
                req->ready = nullptr;
            }
            {
                std::lock_guard<std::mutex> lk(mu);
                arena.release(req->offset);
                admitted_bytes -= req->need;
                --active;
                res.elapsed_ms =
                    std::chrono::duration<double, std::milli>(Clock::now() - req->t_submit).count();
                req->result = res;
                req->status = st;
                req->error = err;
                req->state = ReqState::Done;
                ++n_completed;
            }
            cv_admit.notify_all();
            cv_done.notify_all();
        }
        for (auto& kv : problems) pcg_problem_destroy(kv.second);
        if (stream) (void)hipStreamDestroy(stream);
    }

    pcg_status run(const Request& r, std::map<DescKey, pcg_problem*>& problems, hipStream_t s,
                   pcg_result* res)
    {
        const DescKey key = key_of(r.desc);
        auto it = problems.find(key);
        if (it == problems.end()) {
            pcg_problem* P = nullptr;
            pcg_status st = pcg_problem_create(&r.desc, &P);
            if (st != PCG_OK) return st;
            it = problems.emplace(key, P).first;
        }
        pcg_problem* P = it->second;
        const size_t n = (size_t)P->geom.n;
        char* base = arena_base + r.offset;
        if (r.device_io) {   // b and x live in the caller's device memory
            if (r.ready && hipStreamWaitEvent(s, r.ready, 0) != hipSuccess) {
                pcg::set_error("pcg server: waiting for the producer stream failed");
                return PCG_E_DEVICE;
            }
            pcg_status st = pcg::solve(P, r.b_host, r.x_host, base, r.need, r.opts, 1, res, s);
            if (hipStreamSynchronize(s) != hipSuccess) {
                pcg::set_error("pcg server: stream synchronisation failed");
                return PCG_E_DEVICE;
            }
            return st;
        }
        double* b = reinterpret_cast<double*>(base);
        double* x = reinterpret_cast<double*>(base + al256(8 * n));
        char* ws = base + 2 * al256(8 * n);
        const size_t ws_bytes = r.need - 2 * al256(8 * n);
        if (hipMemcpyAsync(b, r.b_host, 8 * n, hipMemcpyHostToDevice, s) != hipSuccess) {
            pcg::set_error("pcg server: host-to-device copy failed");
            return PCG_E_DEVICE;
        }
        pcg_status st = pcg::solve(P, b, x, ws, ws_bytes, r.opts, 1, res, s);
        if (st != PCG_OK && st != PCG_E_NOCONV && st != PCG_E_BREAKDOWN) return st;
        if (hipMemcpyAsync(r.x_host, x, 8 * n, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            pcg::set_error("pcg server: device-to-host copy failed");
            return PCG_E_DEVICE;
        }
        return st;
    }
};

extern "C" {

size_t pcg_request_bytes(const pcg_problem_desc* desc, const pcg_solve_opts* opts)
{
    if (!desc || !pcg::validate(*desc).empty()) return 0;
    pcg_solve_opts o;
    if (opts) o = *opts;
    else pcg_default_opts(&o);
    const int64_t n = (int64_t)desc->nx * desc->ny * desc->nz;
    return 2 * al256(8 * (size_t)n) + pcg::request_bytes(*desc, o);
}

pcg_status pcg_server_create(const pcg_server_opts* opts, void* arena, size_t arena_bytes,
                             pcg_server** out)
{
    if (!opts || !arena || !out || arena_bytes < 256 || opts->max_active < 1 ||
        opts->max_active > 64 || opts->hbm_budget_bytes == 0) {
        pcg::set_error("pcg_server_create: need opts, an arena of >= 256 bytes, "
                       "1 <= max_active <= 64 and a non-zero budget");
        return PCG_E_INVALID;
    }
    if ((reinterpret_cast<uintptr_t>(arena) & 255u) != 0) {
        pcg::set_error("pcg_server_create: the arena must be 256-byte aligned");
        return PCG_E_INVALID;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        pcg::set_error("pcg_server_create: no HIP device");
        return PCG_E_DEVICE;
    }
    pcg_server* S = new (std::nothrow) pcg_server();
    if (!S) return PCG_E_NOMEM;
    S->opts = *opts;
    S->opts.hbm_budget_bytes = std::min(opts->hbm_budget_bytes, arena_bytes);
    S->device = dev;
    S->arena_base = static_cast<char*>(arena);
    S->arena.reset(arena_bytes);
    try {
        for (int i = 0; i < S->opts.max_active; ++i)
            S->workers.emplace_back([S] { S->worker_main(); });
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stop = true;
        }
        S->cv_admit.notify_all();
        for (auto& t : S->workers) t.join();
        delete S;
        pcg::set_error("pcg_server_create: could not start worker threads");
        return PCG_E_NOMEM;
    }
    *out = S;
    return PCG_OK;
}

static pcg_status submit(pcg_server* S, const pcg_problem_desc* desc, const pcg_solve_opts* opts,
                         const double* b, double* x, bool device_io, hipStream_t producer,
                         uint64_t* ticket)
{
    if (!S || !desc || !b || !x || !ticket) {
        pcg::set_error("pcg_submit: NULL argument");
        return PCG_E_INVALID;
    }
    if (device_io && (((reinterpret_cast<uintptr_t>(b) | reinterpret_cast<uintptr_t>(x)) & 15u) ||
                      static_cast<const void*>(b) == static_cast<const void*>(x))) {
        pcg::set_error("pcg_submit_device: b and x must be distinct 16-byte aligned device arrays");
        return PCG_E_INVALID;
    }
    const std::string err = pcg::validate(*desc);
    if (!err.empty()) {
        pcg::set_error("pcg_submit: " + err);
        return PCG_E_INVALID;
    }
    auto r = std::make_shared<Request>();
    r->desc = *desc;
    if (opts) r->opts = *opts;
    else pcg_default_opts(&r->opts);
    r->opts.x0_zero = 1;        // served solves start from zero (x_host is output only)
    r->opts.profile = 0;
    if (!(r->opts.fused) || r->opts.max_iter < 1 || !(r->opts.rtol >= 0.0)) {
        pcg::set_error("pcg_submit: served solves run the fused iteration with max_iter >= 1");
        return PCG_E_INVALID;
    }
    r->b_host = b;
    r->x_host = x;
    r->device_io = device_io;
    r->need = pcg_request_bytes(desc, &r->opts);
    if (device_io) {   // only the workspace lives in the arena
        r->need = pcg::request_bytes(*desc, r->opts);
        // order the solve after the work already queued on the producer stream
        if (hipEventCreateWithFlags(&r->ready, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(r->ready, producer) != hipSuccess) {
            if (r->ready) (void)hipEventDestroy(r->ready);
            r->ready = nullptr;
            pcg::set_error("pcg_submit_device: could not record the producer stream");
            return PCG_E_DEVICE;
        }
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (r->need > S->opts.hbm_budget_bytes || r->need > S->arena.size()) {
        if (r->ready) (void)hipEventDestroy(r->ready);
        r->ready = nullptr;
        ++S->n_rejected;
        std::ostringstream m;
        m << "pcg_submit: request needs " << r->need << " bytes; budget " << S->opts.hbm_budget_bytes
          << ", arena " << S->arena.size();
        pcg::set_error(m.str());
        return PCG_E_NOMEM;
    }
    r->ticket = S->next_ticket++;
    r->t_submit = Clock::now();
    S->queue.push_back(r);
    S->tickets[r->ticket] = r;
    ++S->n_submitted;
    *ticket = r->ticket;
    S->cv_admit.notify_one();
    return PCG_OK;
}

pcg_status pcg_submit(pcg_server* S, const pcg_problem_desc* desc, const pcg_solve_opts* opts,
                      const double* b_host, double* x_host, uint64_t* ticket)
{
    return submit(S, desc, opts, b_host, x_host, false, nullptr, ticket);
}

pcg_status pcg_submit_device(pcg_server* S, const pcg_problem_desc* desc,
                             const pcg_solve_opts* opts, const double* b_dev, double* x_dev,
                             void* stream, uint64_t* ticket)
{
    return submit(S, desc, opts, b_dev, x_dev, true, static_cast<hipStream_t>(stream), ticket);
}

static pcg_status finish_ticket(pcg_server* S, std::unordered_map<uint64_t, std::shared_ptr<Request>>::iterator it,
                                pcg_result* out)
{
    auto r = it->second;
    if (r->state == ReqState::Cancelled) {
        S->tickets.erase(it);
        return PCG_E_CANCELLED;
    }
    if (out) *out = r->result;
    const pcg_status st = r->status;
    if (!r->error.empty()) pcg::set_error(r->error);   // report in the polling thread
    S->tickets.erase(it);
    return st;
}

pcg_status pcg_poll(pcg_server* S, uint64_t ticket, pcg_result* out)
{
    if (!S) return PCG_E_INVALID;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) {
        pcg::set_error("pcg_poll: unknown ticket");
        return PCG_E_INVALID;
    }
    const ReqState st = it->second->state;
    if (st == ReqState::Queued || st == ReqState::Running) return PCG_E_AGAIN;
    return finish_ticket(S, it, out);
}

pcg_status pcg_wait(pcg_server* S, uint64_t ticket, pcg_result* out)
{
    if (!S) return PCG_E_INVALID;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) {
        pcg::set_error("pcg_wait: unknown ticket");
        return PCG_E_INVALID;
    }
    auto r = it->second;
    S->cv_done.wait(lk, [&] { return r->state == ReqState::Done || r->state == ReqState::Cancelled; });
    it = S->tickets.find(ticket);
    if (it == S->tickets.end()) {   // another thread collected it meanwhile
        pcg::set_error("pcg_wait: ticket collected by another call");
        return PCG_E_INVALID;
    }
    return finish_ticket(S, it, out);
}

pcg_status pcg_cancel(pcg_server* S, uint64_t ticket)
{
    if (!S) return PCG_E_INVALID;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) {
        pcg::set_error("pcg_cancel: unknown ticket");
        return PCG_E_INVALID;
    }
    auto r = it->second;
    if (r->state != ReqState::Queued) {
        pcg::set_error("pcg_cancel: only queued requests can be cancelled");
        return PCG_E_AGAIN;
    }
    for (auto q = S->queue.begin(); q != S->queue.end(); ++q)
        if ((*q)->ticket == ticket) {
            S->queue.erase(q);
            break;
        }
    r->state = ReqState::Cancelled;
    if (r->ready) {
        (void)hipEventDestroy(r->ready);
        r->ready = nullptr;
    }
    ++S->n_cancelled;
    S->cv_admit.notify_all();   // the head may have changed
    S->cv_done.notify_all();
    return PCG_OK;
}

pcg_status pcg_server_query(pcg_server* S, pcg_server_stats* out)
{
    if (!S || !out) return PCG_E_INVALID;
    std::lock_guard<std::mutex> lk(S->mu);
    out->submitted = S->n_submitted;
    out->completed = S->n_completed;
    out->cancelled = S->n_cancelled;
    out->rejected = S->n_rejected;
    out->queued = (int32_t)S->queue.size();
    out->active = S->active;
    out->bytes_in_use = S->admitted_bytes;
    out->peak_bytes_in_use = S->peak_bytes;
    out->peak_active = S->peak_active;
    out->reserved = 0;
    return PCG_OK;
}

void pcg_server_destroy(pcg_server* S)
{
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        for (auto& r : S->queue) {
            r->state = ReqState::Cancelled;
            if (r->ready) {
                (void)hipEventDestroy(r->ready);
                r->ready = nullptr;
            }
            ++S->n_cancelled;
        }
        S->queue.clear();
        S->stop = true;
    }
    S->cv_admit.notify_all();
    S->cv_done.notify_all();
    for (auto& t : S->workers) t.join();
    delete S;
}

}  // extern "C"
