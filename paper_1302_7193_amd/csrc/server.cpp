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
//
// Batched mode (pcg_server_opts.batched = 1): one scheduler thread advances
// every admitted request with shared launches.  Each tick runs, for the
// requests at that stage, the FP64 refinement residual, then K iterations of
// kernels A and B (requests that join start with their first kernel B),
// then the refinement update or exit correction -- every one a single
// multi-request launch over all of them (multi.h), each request keeping its
// own launch shape (the served shape: fixed levels per lane, lanes per column
// n_z / levels), partial sums and solver state.  Requests arriving while
// others run join at the next tick; the ones that finish leave and free their
// memory.  A request's kernels and reduction orders do not depend on which
// others share its launches, so its result is the same alone and in any mix.
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
#include "multi.h"
#include "problem.h"

namespace pcg {

size_t request_bytes(const pcg_problem_desc& d, const pcg_solve_opts& o);
int resolve_precond(const pcg_problem_desc& d, double dx, const pcg_solve_opts& o);
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

// ---------------------------------------------------------- batched mode --

constexpr int kServeK = 4;            // iterations of kernels A and B per tick
// launch tables of a tick (device and pinned host copies, one of each)
enum : int {
    kTabResidual, kTabStart32, kTabStart64, kTabApply32, kTabPrec32, kTabApply64, kTabPrec64,
    kTabUpdate, kTabFixup, kNumTabs
};
constexpr int64_t kServeCap = 2048;   // workgroups per request and kernel

// Lanes per column of the served launch shape: n_z / levels per lane (4 in
// FP32, 2 in FP64), a power of two up to 64; 0 when n_z does not allow it.
int serve_lanes(int nz, int levels)
{
    if (nz % levels) return 0;
    const int L = nz / levels;
    return (L >= 1 && L <= pcg::kWave && (L & (L - 1)) == 0) ? L : 0;
}

pcg::SolverState serve_state(double rtol, double atol, int max_iter, double aux)
{
    pcg::SolverState st;
    std::memset(&st, 0, sizeof(st));
    st.kappa_old = 1.0;
    st.rtol = rtol;
    st.atol = atol;
    st.max_iter = max_iter;
    st.aux = aux;
    st.flag = pcg::kRunning;
    return st;
}

enum class Phase { Residual, InnerStart, InnerRun, Update, Fixup, Done };

// One admitted request in batched mode.  States: the server's device state
// array holds two per slot (index 2*idx: the Krylov solve, 2*idx + 1: the
// refinement); the host mirrors them between launches.
struct BSlot {
    std::shared_ptr<Request> req;
    int idx = 0;
    bool mixed = false;
    Phase phase = Phase::Residual;
    pcg::ColArgs kry{}, res{}, upd{};   // Krylov kernels, FP64 residual, FP64 update
    double* b = nullptr;
    double* x = nullptr;
    int64_t n = 0;
    // refinement bookkeeping, as in the mixed-precision solve
    int k = 0, inner_iters = 0, outer_steps = 0;
    double r0 = 0.0, rn = 0.0, scale = 1.0;
    bool rescaled = false;
    pcg_status stat = PCG_E_NOCONV;
    int launches = 0;
};

}  // namespace

struct pcg_server {
    pcg_server_opts opts{};
    int device = 0;
    // batched mode: slot states and launch tables (device, with pinned mirrors)
    pcg::SolverState* d_states = nullptr;
    pcg::SolverState* h_states = nullptr;
    pcg::MultiTable* d_tables = nullptr;
    pcg::MultiTable* h_tables = nullptr;
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

    void free_batched()
    {
        if (d_states) (void)hipFree(d_states);
        if (d_tables) (void)hipFree(d_tables);
        if (h_states) (void)hipHostFree(h_states);
        if (h_tables) (void)hipHostFree(h_tables);
        d_states = h_states = nullptr;
        d_tables = h_tables = nullptr;
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

    // ------------------------------------------------------ batched mode --

    // Under mu: the head request if it can be admitted into a free slot now.
    std::shared_ptr<Request> try_admit_slot(int free_slots)
    {
        if (free_slots <= 0) return nullptr;
        return try_admit();
    }

    void finish_request(const std::shared_ptr<Request>& req, const pcg_result& res, pcg_status st,
                        const std::string& err)
    {
        std::lock_guard<std::mutex> lk(mu);
        arena.release(req->offset);
        admitted_bytes -= req->need;
        --active;
        pcg_result r = res;
        r.elapsed_ms = std::chrono::duration<double, std::milli>(Clock::now() - req->t_submit).count();
        req->result = r;
        req->status = st;
        req->error = err;
        req->state = ReqState::Done;
        ++n_completed;
    }

    // Sets up slot sl for its admitted request: problem tables, vectors in the
    // arena (or the caller's), launch blocks of the served shape.
    pcg_status setup_slot(BSlot& sl, std::map<DescKey, pcg_problem*>& problems, hipStream_t s)
    {
        const Request& r = *sl.req;
        const DescKey key = key_of(r.desc);
        auto it = problems.find(key);
        if (it == problems.end()) {
            pcg_problem* P = nullptr;
            const pcg_status st = pcg_problem_create(&r.desc, &P);
            if (st != PCG_OK) return st;
            it = problems.emplace(key, P).first;
        }
        pcg_problem* P = it->second;
        sl.n = P->geom.n;
        sl.mixed = r.opts.precision == PCG_PREC_MIXED;
        const size_t n = (size_t)sl.n;
        char* base = arena_base + r.offset;
        if (r.device_io) {
            sl.b = const_cast<double*>(r.b_host);
            sl.x = r.x_host;
            if (r.ready && hipStreamWaitEvent(s, r.ready, 0) != hipSuccess) {
                pcg::set_error("pcg server: waiting for the producer stream failed");
                return PCG_E_DEVICE;
            }
        } else {
            sl.b = reinterpret_cast<double*>(base);
            sl.x = reinterpret_cast<double*>(base + al256(8 * n));
            base += 2 * al256(8 * n);
            if (hipMemcpyAsync(sl.b, r.b_host, 8 * n, hipMemcpyHostToDevice, s) != hipSuccess) {
                pcg::set_error("pcg server: host-to-device copy failed");
                return PCG_E_DEVICE;
            }
        }
        // workspace: the Krylov vectors (r, z, p, q, and u when mixed: the
        // FP64 solve's u is x), then the partial sums -- within the request's
        // arena block, which has room for these and 65536 partial-sum slots
        const size_t ev = sl.mixed ? 4 : 8;
        const int nvec = sl.mixed ? 5 : 4;
        void* vec[5] = {};
        for (int v = 0; v < nvec; ++v) {
            vec[v] = base;
            base += al256(ev * n);
        }
        double* part = reinterpret_cast<double*>(base);
        if ((size_t)(base - (arena_base + r.offset)) + kServeCap * pcg::kRedSlots * sizeof(double) >
            r.need) {
            pcg::set_error("pcg server: a batched request's vectors do not fit its arena block");
            return PCG_E_INVALID;
        }
        pcg::Shape sh;
        pcg::ColArgs a{};
        a.g = P->geom;
        a.red_mode = 1;
        a.part = part;
        // Krylov kernels: FP32 (mixed) or FP64, line preconditioner, z and p
        // trading vectors (the solver's zswap)
        const int Lk = serve_lanes(P->geom.nz, sl.mixed ? pcg::kServeM32 : pcg::kServeM64);
        sh.L = Lk;
        sl.kry = a;
        sl.kry.L = sl.kry.L_b = Lk;
        sl.kry.blocks_per_rhs = sl.kry.bpr_b = std::min(pcg::column_blocks(P->geom, sh), kServeCap);
        sl.kry.vert = sl.mixed ? (const void*)P->d_vert32 : (const void*)P->d_vert64;
        sl.kry.lu = sl.mixed ? (const void*)P->d_lu32 : (const void*)P->d_lu64;
        sl.kry.io0 = sl.mixed ? vec[4] : sl.x;   // u
        sl.kry.io1 = vec[0];                     // r
        sl.kry.io2 = vec[1];                     // z
        sl.kry.io3 = vec[2];                     // p
        sl.kry.io4 = vec[3];                     // q
        sl.kry.in1 = sl.mixed ? vec[0] : sl.b;   // b of the Krylov solve (r32 itself when mixed)
        sl.kry.st = d_states + 2 * sl.idx;
        sl.kry.zswap = 1;
        // FP64 refinement residual and update
        const int L64 = serve_lanes(P->geom.nz, pcg::kServeM64);
        sh.L = L64;
        sl.res = a;
        sl.res.L = sl.res.L_b = L64;
        sl.res.blocks_per_rhs = sl.res.bpr_b = std::min(pcg::column_blocks(P->geom, sh), kServeCap);
        sl.res.vert = P->d_vert64;
        sl.res.lu = P->d_lu64;
        sl.res.in0 = sl.x;
        sl.res.in1 = sl.b;
        sl.res.io0 = sl.x;
        sl.res.out32 = vec[0];                   // r32, the inner right-hand side
        sl.res.st = d_states + 2 * sl.idx + 1;
        sl.upd = sl.res;
        sl.upd.out32 = vec[4];                   // u32
        sl.upd.in0 = vec[1];                     // p32 (in z's vector after the first kernel A)
        sl.upd.st_in = d_states + 2 * sl.idx;
        sl.phase = sl.mixed ? Phase::Residual : Phase::InnerStart;
        return PCG_OK;
    }

    // Launches op over the given slots' blocks from table `tab` (filled and
    // uploaded when `fill`; a table is filled at most once per tick, and
    // every tick ends with a stream synchronisation, so a pinned table is
    // never rewritten while its copy is pending).
    pcg_status launch_op(pcg::MultiOp op, int tab, bool fill, const std::vector<BSlot*>& group,
                         pcg::ColArgs BSlot::*which, hipStream_t s)
    {
        if (group.empty()) return PCG_OK;
        pcg::MultiTable& t = h_tables[tab];
        pcg::MultiTable* dt = d_tables + tab;
        if (fill) {
            t.nslots = (int32_t)group.size();
            int64_t total = 0;
            for (size_t i = 0; i < group.size(); ++i) {
                t.start[i] = total;
                t.args[i] = group[i]->*which;
                total += t.args[i].blocks_per_rhs;
            }
            t.start[group.size()] = total;
            if (hipMemcpyAsync(dt, &t, sizeof(pcg::MultiTable), hipMemcpyHostToDevice, s) !=
                hipSuccess) {
                pcg::set_error("pcg server: launch table upload failed");
                return PCG_E_DEVICE;
            }
        }
        for (BSlot* p : group) ++p->launches;
        if (pcg::multi_launch(op, dt, t.start[t.nslots], t.nslots, s) != hipSuccess) {
            pcg::set_error("pcg server: multi-request launch failed");
            return PCG_E_DEVICE;
        }
        return PCG_OK;
    }

    pcg_status sync_states(hipStream_t s, bool upload)
    {
        const size_t bytes = sizeof(pcg::SolverState) * 2 * pcg::kMaxSlots;
        if (upload) {
            if (hipMemcpyAsync(d_states, h_states, bytes, hipMemcpyHostToDevice, s) != hipSuccess)
                return PCG_E_DEVICE;
            return PCG_OK;
        }
        if (hipMemcpyAsync(h_states, d_states, bytes, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return PCG_E_DEVICE;
        return PCG_OK;
    }

    void scheduler_main()
    {
        (void)hipSetDevice(device);
        hipStream_t stream = nullptr;
        const bool have_stream = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess;
        std::map<DescKey, pcg_problem*> problems;
        const int max_slots = std::min(opts.max_active, pcg::kMaxSlots);
        std::vector<BSlot> slots;
        std::vector<int> free_idx;
        for (int i = max_slots - 1; i >= 0; --i) free_idx.push_back(i);
        auto fail_all = [&](const std::string& why) {
            for (BSlot& sl : slots) finish_request(sl.req, pcg_result{}, PCG_E_DEVICE, why);
            slots.clear();
            free_idx.clear();
            for (int i = max_slots - 1; i >= 0; --i) free_idx.push_back(i);
        };
        for (;;) {
            // admit whatever fits (waiting only when nothing is running)
            {
                std::unique_lock<std::mutex> lk(mu);
                if (slots.empty())
                    cv_admit.wait(lk, [&] { return stop || !queue.empty(); });
                if (stop && slots.empty()) break;
                std::shared_ptr<Request> req;
                while (!stop && (req = try_admit_slot((int)free_idx.size())) != nullptr) {
                    BSlot sl;
                    sl.req = req;
                    sl.idx = free_idx.back();
                    free_idx.pop_back();
                    slots.push_back(sl);
                }
            }
            if (!have_stream) {
                fail_all("pcg server: could not create the scheduler stream");
                continue;
            }
            for (BSlot& sl : slots) {
                if (sl.kry.st) continue;   // set up already
                const pcg_status st = setup_slot(sl, problems, stream);
                if (st != PCG_OK) {
                    char buf[512];
                    pcg_last_error(buf, sizeof(buf));
                    sl.stat = st;
                    sl.phase = Phase::Done;
                    sl.req->error = buf;
                }
            }
            if (tick(slots, stream) != PCG_OK) {
                fail_all("pcg server: device error in a multi-request launch");
                continue;
            }
            // retire finished requests
            bool copied = false;
            for (BSlot& sl : slots)
                if (sl.phase == Phase::Done && sl.kry.st && !sl.req->device_io) {
                    if (hipMemcpyAsync(sl.req->x_host, sl.x, 8 * (size_t)sl.n, hipMemcpyDeviceToHost,
                                       stream) != hipSuccess)
                        sl.stat = PCG_E_DEVICE;
                    copied = true;
                }
            if (copied && hipStreamSynchronize(stream) != hipSuccess) {
                fail_all("pcg server: device-to-host copy failed");
                continue;
            }
            for (auto it = slots.begin(); it != slots.end();) {
                if (it->phase != Phase::Done) {
                    ++it;
                    continue;
                }
                pcg_result res{};
                const pcg::SolverState& hk = h_states[2 * it->idx];
                res.status = it->stat;
                res.launches = it->launches;
                res.preconditioner = PCG_PRECOND_LINE;
                if (it->mixed) {
                    res.iterations = it->inner_iters;
                    res.outer_iterations = it->outer_steps;
                    res.r0_norm = it->r0;
                    res.rel_res_recursive = it->r0 > 0 ? it->rn / it->r0 : 0.0;
                    res.rel_res_true = res.rel_res_recursive;
                } else {
                    res.iterations = hk.iter;
                    res.r0_norm = hk.r0norm;
                    res.rel_res_recursive = hk.r0norm > 0 ? hk.rnorm / hk.r0norm : 0.0;
                    res.rel_res_true = -1.0;
                }
                if (it->req->ready) {
                    (void)hipEventDestroy(it->req->ready);
                    it->req->ready = nullptr;
                }
                const std::string err = it->req->error;
                finish_request(it->req, res, it->stat, it->stat == PCG_OK || it->stat == PCG_E_NOCONV ||
                                                           it->stat == PCG_E_BREAKDOWN ? std::string() : err);
                free_idx.push_back(it->idx);
                it = slots.erase(it);
            }
            cv_admit.notify_all();
            cv_done.notify_all();
        }
        for (auto& kv : problems) pcg_problem_destroy(kv.second);
        if (stream) (void)hipStreamDestroy(stream);
    }

    // One tick: residuals, K iterations, updates / exit corrections of the
    // admitted requests at those stages.
    pcg_status tick(std::vector<BSlot>& slots, hipStream_t s)
    {
        using pcg::MultiOp;
        std::vector<BSlot*> grp;
        // FP64 refinement residuals
        for (BSlot& sl : slots)
            if (sl.phase == Phase::Residual) {
                pcg::SolverState st = serve_state(sl.req->opts.rtol, sl.req->opts.atol, 0, sl.scale);
                st.iter = 0;
                h_states[2 * sl.idx + 1] = st;
                sl.res.x0_zero = (sl.k == 0) ? 1 : 0;   // x0 = 0: x not read yet
                grp.push_back(&sl);
            }
        if (!grp.empty()) {
            if (sync_states(s, true) != PCG_OK ||
                launch_op(MultiOp::Residual64, kTabResidual, true, grp, &BSlot::res, s) ||
                sync_states(s, false) != PCG_OK)
                return PCG_E_DEVICE;
            for (BSlot* p : grp) residual_done(*p, s);
            // a zero start that stops here has written nothing to x: x = 0
            for (BSlot* p : grp)
                if (p->phase == Phase::Done && p->k == 0 &&
                    hipMemsetAsync(p->x, 0, 8 * (size_t)p->n, s) != hipSuccess)
                    return PCG_E_DEVICE;
        }
        // Krylov iterations: requests that start take their first kernel B
        std::vector<BSlot*> start32, start64, run32, run64;
        for (BSlot& sl : slots) {
            if (sl.phase == Phase::InnerStart) {
                const pcg_solve_opts& o = sl.req->opts;
                pcg::SolverState st = sl.mixed
                    ? serve_state(o.inner_rtol, 0.0, std::max(1, o.max_iter - sl.inner_iters), 1.0)
                    : serve_state(o.rtol, o.atol, o.max_iter, 1.0);
                st.zero_start = 1;
                h_states[2 * sl.idx] = st;
                (sl.mixed ? start32 : start64).push_back(&sl);
                sl.phase = Phase::InnerRun;
            }
            if (sl.phase == Phase::InnerRun) (sl.mixed ? run32 : run64).push_back(&sl);
        }
        if (!run32.empty() || !run64.empty()) {
            if (sync_states(s, true) != PCG_OK ||
                launch_op(MultiOp::PrecF32, kTabStart32, true, start32, &BSlot::kry, s) ||
                launch_op(MultiOp::PrecF64, kTabStart64, true, start64, &BSlot::kry, s))
                return PCG_E_DEVICE;
            for (int i = 0; i < kServeK; ++i)
                if (launch_op(MultiOp::ApplyF32, kTabApply32, i == 0, run32, &BSlot::kry, s) ||
                    launch_op(MultiOp::PrecF32, kTabPrec32, i == 0, run32, &BSlot::kry, s) ||
                    launch_op(MultiOp::ApplyF64, kTabApply64, i == 0, run64, &BSlot::kry, s) ||
                    launch_op(MultiOp::PrecF64, kTabPrec64, i == 0, run64, &BSlot::kry, s))
                    return PCG_E_DEVICE;
            if (sync_states(s, false) != PCG_OK) return PCG_E_DEVICE;
            for (BSlot* p : run32)
                if (h_states[2 * p->idx].flag != pcg::kRunning) p->phase = Phase::Update;
            for (BSlot* p : run64)
                if (h_states[2 * p->idx].flag != pcg::kRunning) p->phase = Phase::Fixup;
        }
        // refinement updates (folding in the exit correction) and FP64 exit corrections
        std::vector<BSlot*> upd, fix;
        for (BSlot& sl : slots) {
            if (sl.phase == Phase::Update) {
                h_states[2 * sl.idx + 1] = serve_state(sl.req->opts.rtol, sl.req->opts.atol, 0, sl.scale);
                sl.upd.x0_zero = (sl.k == 0) ? 1 : 0;
                upd.push_back(&sl);
            } else if (sl.phase == Phase::Fixup) {
                fix.push_back(&sl);
            }
        }
        if (!upd.empty() || !fix.empty()) {
            if (sync_states(s, true) != PCG_OK ||
                launch_op(MultiOp::Update64, kTabUpdate, true, upd, &BSlot::upd, s) ||
                launch_op(MultiOp::FixupF64, kTabFixup, true, fix, &BSlot::kry, s))
                return PCG_E_DEVICE;
            for (BSlot* p : upd) update_done(*p);
            for (BSlot* p : fix) {
                const pcg::SolverState& hk = h_states[2 * p->idx];
                p->stat = hk.flag == pcg::kConverged ? PCG_OK
                          : hk.flag == pcg::kBreakdown ? PCG_E_BREAKDOWN : PCG_E_NOCONV;
                p->phase = Phase::Done;
            }
            if (sync_states(s, false) != PCG_OK) return PCG_E_DEVICE;
        }
        return PCG_OK;
    }

    // After a refinement residual: the exit test, or the next inner solve
    // (the bookkeeping of the mixed-precision solve, per request).
    void residual_done(BSlot& sl, hipStream_t)
    {
        const pcg_solve_opts& o = sl.req->opts;
        const pcg::SolverState& ho = h_states[2 * sl.idx + 1];
        sl.rn = ho.rnorm;
        if (sl.k == 0 && !sl.rescaled) sl.r0 = sl.rn;
        if (!std::isfinite(sl.rn)) {
            sl.stat = PCG_E_BREAKDOWN;
            sl.phase = Phase::Done;
        } else if (sl.r0 == 0.0 || sl.rn / sl.r0 < o.rtol || sl.rn < o.atol) {
            sl.stat = PCG_OK;
            sl.phase = Phase::Done;
        } else if (sl.k >= o.max_outer || sl.inner_iters >= o.max_iter) {
            sl.stat = PCG_E_NOCONV;
            sl.phase = Phase::Done;
        } else if (sl.k == 0 && !sl.rescaled && (sl.rn > 1e20 || sl.rn < 1e-20)) {
            sl.scale = 1.0 / sl.rn;   // keep the FP32 residual near unit size: redo it
            sl.rescaled = true;
        } else {
            sl.phase = Phase::InnerStart;
        }
    }

    void update_done(BSlot& sl)
    {
        const pcg::SolverState& hi = h_states[2 * sl.idx];
        sl.inner_iters += hi.iter;
        sl.outer_steps += 1;
        sl.k += 1;
        if (hi.flag == pcg::kBreakdown && hi.iter == 0) {
            sl.stat = PCG_E_BREAKDOWN;
            sl.phase = Phase::Done;
            return;
        }
        const double red = hi.r0norm > 0 ? hi.rnorm / hi.r0norm : 1.0;
        const double est = sl.rn * std::max(red, 1e-30);
        if (std::isfinite(est) && est > 0) sl.scale = 1.0 / est;
        sl.phase = Phase::Residual;
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
    if (opts->batched != 0 && opts->batched != 1) {
        pcg::set_error("pcg_server_create: batched must be 0 or 1");
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
    if (S->opts.batched) {   // slot states and launch tables, device and pinned host copies
        const size_t sb = sizeof(pcg::SolverState) * 2 * pcg::kMaxSlots;
        const size_t tb = sizeof(pcg::MultiTable) * kNumTabs;
        if (hipMalloc((void**)&S->d_states, sb) != hipSuccess ||
            hipMalloc((void**)&S->d_tables, tb) != hipSuccess ||
            hipHostMalloc((void**)&S->h_states, sb, 0) != hipSuccess ||
            hipHostMalloc((void**)&S->h_tables, tb, 0) != hipSuccess) {
            S->free_batched();
            delete S;
            pcg::set_error("pcg_server_create: could not allocate the batched-mode tables");
            return PCG_E_NOMEM;
        }
        std::memset(S->h_states, 0, sb);
        std::memset(S->h_tables, 0, tb);
    }
    try {
        if (S->opts.batched) {
            S->workers.emplace_back([S] { S->scheduler_main(); });
        } else {
            for (int i = 0; i < S->opts.max_active; ++i)
                S->workers.emplace_back([S] { S->worker_main(); });
        }
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stop = true;
        }
        S->cv_admit.notify_all();
        for (auto& t : S->workers) t.join();
        S->free_batched();
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
    if (S->opts.batched) {   // what the multi-request kernels cover
        const pcg_problem_desc& d = *desc;
        const bool line = pcg::resolve_precond(d, d.dx, r->opts) == PCG_PRECOND_LINE;
        const int lv = r->opts.precision == PCG_PREC_MIXED ? pcg::kServeM32 : pcg::kServeM64;
        if (!line || !serve_lanes(d.nz, lv) || !serve_lanes(d.nz, pcg::kServeM64)) {
            pcg::set_error("pcg_submit: a batched server runs the line preconditioner on grids "
                           "with n_z = 4, 8, 16, 32, 64 or 128");
            return PCG_E_INVALID;
        }
        r->opts.preconditioner = PCG_PRECOND_LINE;
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
    S->free_batched();
    delete S;
}

}  // extern "C"
