// Solve drivers of libpcg.
//
// Fused iteration (Alg. InterleavedPCG): after the start-up kernels the host
// issues chunks of K iterations -- K x (kernel A, kernel B) and one exit
// correction -- and reads the device flags once per chunk.  Every kernel
// returns at once when the flag of its right-hand side is set, so a chunk
// that overshoots the exit costs only empty launches.  With an adaptive
// chunk (K = the previous solve's iteration count) a repeated solve issues
// exactly the launches it needs.  Chunks are built once as HIP graphs
// (explicit kernel nodes) and replayed.
//
// Mixed precision: FP64 residual r = b - A x (scaled to FP32), an FP32 inner
// solve of A d = r to a relative tolerance, FP64 update x += d / scale,
// repeated until the FP64 residual meets the tolerance.  The inner solve's
// exit correction d = u + alpha p is folded into the update (no separate
// pass over the FP32 vectors).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <sstream>

#include "problem.h"

namespace pcg {

namespace {

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

int64_t blas_blocks(int64_t n) { return std::max<int64_t>(1, std::min<int64_t>(2048, (n / 2 + kBlock - 1) / kBlock)); }

}  // namespace

int64_t blocks_per_rhs(const pcg_problem* P, int dtype)
{
    const Tuning& t = P->tune[dtype];
    return std::max<int64_t>(1, std::min(t.block_cap, column_blocks(P->geom, t.shape)));
}

int64_t blocks_per_rhs_b(const pcg_problem* P, int dtype)
{
    const Tuning& t = P->tune[dtype];
    return std::max<int64_t>(1, std::min(t.block_cap_b, column_blocks(P->geom, t.shape_b)));
}

namespace {

struct Layout {
    size_t r = 0, z = 0, p = 0, q = 0;           // FP64 vectors
    size_t r32 = 0, z32 = 0, p32 = 0, q32 = 0, u32 = 0;
    size_t part = 0, st = 0, st_o = 0;
    // multigrid: r, t, z of coarse level l at mg_r[l], mg_t[l], mg_z[l]; the
    // fine level uses r and z of the iteration and its own t at mg_t[0]
    size_t mg_r[32] = {}, mg_t[32] = {}, mg_z[32] = {};
    int mg_levels = 1;
    size_t total = 0;
};

// Workspace layout.  `slots`: partial-sum slots per right-hand side (the
// largest workgroup count any kernel of the solve may use).
Layout plan_n(int64_t cells, const pcg_solve_opts& o, int64_t nrhs, int64_t slots)
{
    Layout w;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += al256(bytes);
        return at;
    };
    const size_t n = (size_t)cells * (size_t)nrhs;
    if (o.precision == PCG_PREC_MIXED) {
        w.r32 = take(4 * n);
        w.z32 = take(4 * n);
        w.p32 = take(4 * n);
        w.q32 = take(4 * n);
        w.u32 = take(4 * n);
    } else {
        w.r = take(8 * n);
        w.z = take(8 * n);
        w.p = take(8 * n);
        w.q = take(8 * n);
    }
    const int64_t nb = std::max(slots, blas_blocks(cells));
    w.part = take((size_t)nrhs * nb * kRedSlots * sizeof(double));
    w.st = take((size_t)nrhs * sizeof(SolverState));
    w.st_o = take((size_t)nrhs * sizeof(SolverState));
    w.total = off;
    return w;
}

}  // namespace

// The preconditioner PCG_PRECOND_AUTO stands for (see include/pcg.h), from
// the descriptor and a representative x width.
int resolve_precond(const pcg_problem_desc& d, double dx, const pcg_solve_opts& o)
{
    if (o.preconditioner != PCG_PRECOND_AUTO) return o.preconditioner;
    if (!o.fused) return PCG_PRECOND_LINE;
    const double dz = d.height / d.nz;
    const double gamma2 = d.k_h > 0.0 ? (d.k_v / (dz * dz)) / (d.k_h / (dx * dx)) : 1e300;
    const int64_t n = (int64_t)d.nx * d.ny * d.nz;
    const bool coarsens = d.nx % 2 == 0 && d.ny % 2 == 0 && d.nx / 2 >= kMgMinCells &&
                          d.ny / 2 >= kMgMinCells;
    if (gamma2 <= 300.0 && n >= (int64_t(1) << 22) && coarsens) return PCG_PRECOND_MG;
    const bool red_black = !((d.bc_x == PCG_BC_PERIODIC && d.nx % 2) ||
                             (d.bc_y == PCG_BC_PERIODIC && d.ny % 2));
    if (gamma2 <= 1e4 && red_black) return PCG_PRECOND_RBGS;
    return PCG_PRECOND_LINE;
}

// The options with AUTO resolved for problem P.
pcg_solve_opts resolved_opts(const pcg_problem* P, const pcg_solve_opts& o)
{
    pcg_solve_opts r = o;
    double dx = P->desc.dx;
    if (P->d_hgeo) {   // stretched: the mean x width
        double sum = 0.0;
        for (int i = 0; i < P->desc.nx; ++i) sum += P->hgeo[i];
        dx = sum / P->desc.nx;
    }
    r.preconditioner = resolve_precond(P->desc, dx, o);
    return r;
}

// Multigrid levels a solve with these options uses (1: the fine level only).
int mg_levels_used(const pcg_problem* P, int requested)
{
    const int all = 1 + (int)P->mg.size();
    return requested > 0 ? std::min(requested, all) : all;
}

const Geom& level_geom(const pcg_problem* P, int l) { return l == 0 ? P->geom : P->mg[l - 1].g; }

namespace {

// Vectors of the multigrid preconditioner appended to w (elements of `elem`
// bytes, nrhs right-hand sides): t of the fine level, r, t, z of the others.
void plan_mg(const pcg_problem* P, int levels, int64_t nrhs, size_t elem, Layout& w)
{
    w.mg_levels = levels;
    w.mg_t[0] = w.total;
    w.total += al256(elem * (size_t)P->geom.n * (size_t)nrhs);
    for (int l = 1; l < levels; ++l) {
        const size_t bytes = al256(elem * (size_t)level_geom(P, l).n * (size_t)nrhs);
        w.mg_r[l] = w.total;
        w.mg_t[l] = w.total + bytes;
        w.mg_z[l] = w.total + 2 * bytes;
        w.total += 3 * bytes;
    }
}

// With the problem's current tunings (a workspace sized before a tuning
// change may be too small afterwards; pcg_solve then reports PCG_E_NOMEM).
Layout plan(const pcg_problem* P, const pcg_solve_opts& o0, int64_t nrhs)
{
    const pcg_solve_opts o = resolved_opts(P, o0);
    int64_t slots = 1;
    for (int d = 0; d < 2; ++d)
        slots = std::max({slots, blocks_per_rhs(P, d), blocks_per_rhs_b(P, d)});
    Layout w = plan_n(P->geom.n, o, nrhs, slots);
    if (o.preconditioner == PCG_PRECOND_MG)
        plan_mg(P, mg_levels_used(P, o.mg_levels), nrhs,
                o.precision == PCG_PREC_MIXED ? sizeof(float) : sizeof(double), w);
    return w;
}

std::string hip_msg(hipError_t e, const char* what)
{
    std::ostringstream m;
    m << what << ": " << hipGetErrorName(e) << " (" << hipGetErrorString(e) << ")";
    return m.str();
}

#define PCG_HIP(call, what)                                       \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) {                                   \
            set_error(hip_msg(e_, what));                         \
            return PCG_E_DEVICE;                                  \
        }                                                         \
    } while (0)

pcg_status ensure_pinned(pcg_problem* P, int64_t nrhs)
{
    if (P->pinned_cap >= nrhs) return PCG_OK;
    if (P->pinned_states) (void)hipHostFree(P->pinned_states);
    P->pinned_states = nullptr;
    P->pinned_cap = 0;
    PCG_HIP(hipHostMalloc((void**)&P->pinned_states, sizeof(SolverState) * (size_t)nrhs, 0),
            "hipHostMalloc(solver states)");
    P->pinned_cap = nrhs;
    return PCG_OK;
}

SolverState fresh_state(double rtol, double atol, int max_iter, double aux)
{
    SolverState s;
    std::memset(&s, 0, sizeof(s));
    s.alpha = 0.0;
    s.beta = 0.0;
    s.kappa_old = 1.0;
    s.rtol = rtol;
    s.atol = atol;
    s.max_iter = max_iter;
    s.aux = aux;
    s.flag = kRunning;
    return s;
}

pcg_status upload_states(pcg_problem* P, SolverState* dev, const SolverState* host, int64_t nrhs,
                         hipStream_t s)
{
    if (ensure_pinned(P, nrhs) != PCG_OK) return PCG_E_DEVICE;
    // the pinned staging buffer is also the read-back target: wait for any
    // copy still in flight on this stream before overwriting it
    PCG_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    std::memcpy(P->pinned_states, host, sizeof(SolverState) * (size_t)nrhs);
    PCG_HIP(hipMemcpyAsync(dev, P->pinned_states, sizeof(SolverState) * (size_t)nrhs,
                           hipMemcpyHostToDevice, s),
            "hipMemcpyAsync(states H2D)");
    PCG_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    return PCG_OK;
}

pcg_status read_states(pcg_problem* P, const SolverState* dev, SolverState* host, int64_t nrhs,
                       hipStream_t s)
{
    if (ensure_pinned(P, nrhs) != PCG_OK) return PCG_E_DEVICE;
    PCG_HIP(hipMemcpyAsync(P->pinned_states, dev, sizeof(SolverState) * (size_t)nrhs,
                           hipMemcpyDeviceToHost, s),
            "hipMemcpyAsync(states D2H)");
    PCG_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    std::memcpy(host, P->pinned_states, sizeof(SolverState) * (size_t)nrhs);
    return PCG_OK;
}

pcg_status ensure_events(pcg_problem* P, size_t count)
{
    // timing only: no system-scope fence (and its cache write-back) when
    // an event is recorded; results are read after a stream synchronisation
    while (P->events.size() < count) {
        hipEvent_t e;
        PCG_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence), "hipEventCreate");
        P->events.push_back(e);
    }
    return PCG_OK;
}

template <typename T>
pcg_status launch(Kind k, const ColArgs& a, int64_t nrhs, hipStream_t s, int& count)
{
    hipError_t e = launch_column<T>(k, a, nrhs, s);
    if (e != hipSuccess) {
        set_error(hip_msg(e, "kernel launch"));
        return PCG_E_DEVICE;
    }
    ++count;
    return PCG_OK;
}

// A sequence of column-kernel launches (each main kernel followed by its
// finalize launch when it has one).
struct Phase {
    std::vector<KernelLaunch> k;
    std::vector<char> fin;     // launch i is a finalize launch
    size_t last_main = 0;      // index of the last main kernel
    int mains = 0;
};

template <typename T>
bool add_kind(Phase& ph, Kind kind, const ColArgs& a, int64_t nrhs)
{
    KernelLaunch l[2];
    const int n = column_launches<T>(kind, a, nrhs, l);
    if (n < 1) return false;
    ph.last_main = ph.k.size();
    ++ph.mains;
    for (int i = 0; i < n; ++i) {
        ph.k.push_back(l[i]);
        ph.fin.push_back(i == 1);
    }
    return true;
}

pcg_status issue_phase(const Phase& ph, hipStream_t s, int& count)
{
    for (const KernelLaunch& l : ph.k) {
        const hipError_t e = issue(l, s);
        if (e != hipSuccess) {
            set_error(hip_msg(e, "kernel launch"));
            return PCG_E_DEVICE;
        }
    }
    count += ph.mains;
    return PCG_OK;
}

// Argument block of multigrid level l: its geometry, tables and launch sizes.
ColArgs level_args(const pcg_problem* P, int dtype, const ColArgs& a, int l)
{
    ColArgs x = a;
    if (l > 0) {
        const MgLevel& m = P->mg[l - 1];
        x.g = m.g;
        x.lu = dtype == PCG_F64 ? (const void*)m.d_lu64 : (const void*)m.d_lu32;
        x.hgeo = m.d_hgeo;
    }
    const Tuning& t = P->tune[dtype];
    x.blocks_per_rhs = std::max<int64_t>(1, std::min(t.block_cap, column_blocks(x.g, t.shape)));
    x.bpr_b = std::max<int64_t>(1, std::min(t.block_cap_b, column_blocks(x.g, t.shape_b)));
    x.omega = kMgOmega;
    return x;
}

// Vectors of a V-cycle: per level the residual r, the pre-smoothed t and the
// result z.
struct MgVecs {
    void* r[32];
    void* t[32];
    void* z[32];
};

static_assert((kMgCoarseSweeps - 1) % 2 == 1, "coarsest sweeps must end in z");

// One V-cycle over `levels` levels as kernel launches.  fused: level 0 starts
// with kernel B's update of r (a carries b, r, q and the solver state) and
// its last sweep ends kernel B (reductions, exit test, beta).
template <typename T>
bool mg_phase(const pcg_problem* P, int dtype, const ColArgs& a, int64_t nrhs, int levels,
              const MgVecs& v, bool fused, Phase& ph)
{
    ColArgs x = level_args(P, dtype, a, 0);
    x.io2 = v.t[0];
    if (!fused) x.in0 = v.r[0];
    if (!add_kind<T>(ph, fused ? Kind::MgPreFused : Kind::MgPre, x, nrhs)) return false;
    for (int l = 0; l + 1 < levels; ++l) {
        ColArgs y = level_args(P, dtype, a, l + 1);
        y.g2 = level_geom(P, l);
        y.hgeo2 = l == 0 ? P->d_hgeo : P->mg[l - 1].d_hgeo;
        y.in0 = v.r[l];
        y.in1 = v.t[l];
        y.io0 = v.r[l + 1];
        if (!add_kind<T>(ph, Kind::MgRestrict, y, nrhs)) return false;
        ColArgs z = level_args(P, dtype, a, l + 1);
        z.in0 = v.r[l + 1];
        z.io2 = v.t[l + 1];
        if (!add_kind<T>(ph, Kind::MgPre, z, nrhs)) return false;
    }
    const int lc = levels - 1;   // coarsest: sweeps alternate t -> z -> t -> z
    const int sweeps = kMgCoarseSweeps - 1;
    for (int k = 0; k < sweeps; ++k) {
        ColArgs y = level_args(P, dtype, a, lc);
        y.in0 = v.r[lc];
        y.io3 = k % 2 == 0 ? v.t[lc] : v.z[lc];
        y.io2 = k % 2 == 0 ? v.z[lc] : v.t[lc];
        const bool final = fused && lc == 0 && k == sweeps - 1;
        if (!add_kind<T>(ph, final ? Kind::MgSmoothFinal : Kind::MgSmooth, y, nrhs)) return false;
    }
    for (int l = lc - 1; l >= 0; --l) {
        ColArgs y = level_args(P, dtype, a, l);
        y.g2 = level_geom(P, l + 1);
        y.in0 = v.r[l];
        y.io3 = v.t[l];
        y.io2 = v.z[l];
        y.in1 = v.z[l + 1];
        const bool final = fused && l == 0;
        if (!add_kind<T>(ph, final ? Kind::MgPostFinal : Kind::MgPost, y, nrhs)) return false;
    }
    return true;
}

// Kernel B's work in the fused iteration: one kernel with the line
// preconditioner, or the V-cycle with the multigrid preconditioner (its
// vectors in the workspace; q must survive until the next kernel A).
template <typename T>
pcg_status b_phase(const pcg_problem* P, int dtype, const ColArgs& a, int64_t nrhs,
                   const pcg_solve_opts& o, char* ws, const Layout& w, Phase& ph)
{
    bool ok;
    if (o.preconditioner == PCG_PRECOND_RBGS) {
        ColArgs x = a;
        x.in0 = a.io1;   // the later half-sweeps read r
        ok = add_kind<T>(ph, Kind::RbFirstFused, a, nrhs) && add_kind<T>(ph, Kind::RbBlack, x, nrhs) &&
             add_kind<T>(ph, Kind::RbRedFinal, x, nrhs);
    } else if (o.preconditioner != PCG_PRECOND_MG) {
        ok = add_kind<T>(ph, Kind::FusedPrec, a, nrhs);
    } else {
        MgVecs v{};
        v.r[0] = a.io1;
        v.t[0] = ws + w.mg_t[0];
        v.z[0] = a.io2;
        for (int l = 1; l < w.mg_levels; ++l) {
            v.r[l] = ws + w.mg_r[l];
            v.t[l] = ws + w.mg_t[l];
            v.z[l] = ws + w.mg_z[l];
        }
        ok = mg_phase<T>(P, dtype, a, nrhs, w.mg_levels, v, true, ph);
    }
    if (!ok) {
        set_error("no kernel for this shape (internal)");
        return PCG_E_DEVICE;
    }
    return PCG_OK;
}

// One chunk of the fused iteration: K x (A, B) and the exit correction
// (unless the caller folds it into its own next kernel).  In the first chunk
// of a solve the first kernel A is its first-launch kernel.
template <typename T>
pcg_status issue_chunk(const ColArgs& a, const Phase& bph, int64_t nrhs, int K, bool first,
                       bool fixup, hipStream_t s, int& count)
{
    for (int i = 0; i < K; ++i) {
        const Kind ka = (first && i == 0) ? Kind::FusedApplyFirst : Kind::FusedApply;
        if (launch<T>(ka, a, nrhs, s, count) != PCG_OK) return PCG_E_DEVICE;
        if (issue_phase(bph, s, count) != PCG_OK) return PCG_E_DEVICE;
    }
    return fixup ? launch<T>(Kind::Fixup, a, nrhs, s, count) : PCG_OK;
}

uint64_t bits(double v)
{
    uint64_t u;
    std::memcpy(&u, &v, sizeof(u));
    return u;
}

uint64_t bits(const void* p) { return static_cast<uint64_t>(reinterpret_cast<uintptr_t>(p)); }

void key_geom(GraphKey& k, const Geom& g)
{
    k.insert(k.end(), {uint64_t(uint32_t(g.nx)), uint64_t(uint32_t(g.ny)), uint64_t(uint32_t(g.nz)),
                       uint64_t(uint32_t(g.nzp)), uint64_t(uint32_t(g.per_x)),
                       uint64_t(uint32_t(g.per_y)), uint64_t(g.nh), uint64_t(g.n), bits(g.area),
                       bits(g.ax), bits(g.ay)});
}

// Every field of one kernel node of a graph chunk, for its cache key.
void key_launch(GraphKey& k, const KernelLaunch& l)
{
    const ColArgs& a = l.args;
    k.insert(k.end(), {bits(l.func), l.grid.x, l.grid.y, l.grid.z, l.block.x, l.block.y, l.block.z});
    key_geom(k, a.g);
    key_geom(k, a.g2);
    k.insert(k.end(), {uint64_t(uint32_t(a.L)), uint64_t(a.blocks_per_rhs), uint64_t(uint32_t(a.L_b)),
                       uint64_t(a.bpr_b), bits(a.vert), bits(a.lu), bits(a.in0), bits(a.in1),
                       bits(a.io0), bits(a.io1), bits(a.io2), bits(a.io3), bits(a.io4),
                       bits(a.out32), bits(a.st), bits(a.part), uint64_t(uint32_t(a.red_mode)),
                       uint64_t(uint32_t(a.x0_zero)), bits(a.hgeo), bits(a.hgeo2), bits(a.omega),
                       uint64_t(uint32_t(a.zswap)), bits(a.st_in)});
}

// The chunk as an explicitly built HIP graph (kernel nodes in sequence).  No
// stream capture is involved, so building is independent of what other host
// threads do with their streams.
// profiled: event record nodes around every kernel A (events
// P->gevents[4i], [4i+1] for iteration i) and, when 1, kernel B's launches up
// to its last main kernel ([4i+2], [4i+3]); 2: kernel A only.
// first: the chunk that starts a solve (its first kernel A is the
// first-launch kernel).
template <typename T>
pcg_status chunk_graph(pcg_problem* P, const ColArgs& a, const Phase& bph,
                       int64_t nrhs, int K, bool first, bool fixup, int profiled,
                       hipGraphExec_t* out)
{
    if (profiled) {
        while (P->gevents.size() < 4 * (size_t)K) {
            hipEvent_t e;
            PCG_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence), "hipEventCreate");
            P->gevents.push_back(e);
        }
    }
    // kernel launches in order; event e is recorded before launch i when
    // marks holds (i, e) (i == seq.size(): after the last)
    std::vector<KernelLaunch> seq;
    std::vector<std::pair<size_t, hipEvent_t>> marks;
    auto add = [&](Kind k) -> bool {
        KernelLaunch l[2];
        const int n = column_launches<T>(k, a, nrhs, l);
        for (int i = 0; i < n; ++i) seq.push_back(l[i]);
        return n > 0;
    };
    for (int i = 0; i < K; ++i) {
        const size_t a_main = seq.size();
        if (profiled) marks.emplace_back(a_main, P->gevents[4 * i]);
        if (!add((first && i == 0) ? Kind::FusedApplyFirst : Kind::FusedApply)) {
            set_error("graph: no kernel for this shape (internal)");
            return PCG_E_DEVICE;
        }
        if (profiled) marks.emplace_back(a_main + 1, P->gevents[4 * i + 1]);   // before its finalize
        const size_t b0 = seq.size();
        if (profiled == 1) marks.emplace_back(b0, P->gevents[4 * i + 2]);
        seq.insert(seq.end(), bph.k.begin(), bph.k.end());
        if (profiled == 1) marks.emplace_back(b0 + bph.last_main + 1, P->gevents[4 * i + 3]);
    }
    if (fixup && !add(Kind::Fixup)) {
        set_error("graph: no kernel for this shape (internal)");
        return PCG_E_DEVICE;
    }
    GraphKey key;
    key.reserve(1 + seq.size() * 48);
    key.push_back((uint64_t)profiled);
    for (const KernelLaunch& l : seq) key_launch(key, l);
    const uint64_t now = ++P->graph_clock;
    auto it = P->graphs.find(key);
    if (it != P->graphs.end()) {
        it->second.last_use = now;
        *out = it->second.exec;
        return PCG_OK;
    }
    // bounded cache: drop the least recently replayed graph (every replay of
    // this problem has completed: solves end with a stream synchronisation)
    if (P->graphs.size() >= kMaxGraphs) {
        auto lru = P->graphs.begin();
        for (auto j = P->graphs.begin(); j != P->graphs.end(); ++j)
            if (j->second.last_use < lru->second.last_use) lru = j;
        (void)hipGraphExecDestroy(lru->second.exec);
        P->graphs.erase(lru);
    }
    hipGraph_t graph = nullptr;
    PCG_HIP(hipGraphCreate(&graph, 0), "hipGraphCreate");
    hipGraphNode_t prev = nullptr;
    size_t next_mark = 0;
    auto add_marks = [&](size_t at) -> pcg_status {
        for (; next_mark < marks.size() && marks[next_mark].first == at; ++next_mark) {
            hipGraphNode_t node = nullptr;
            const hipError_t e = hipGraphAddEventRecordNode(&node, graph, prev ? &prev : nullptr,
                                                            prev ? 1 : 0, marks[next_mark].second);
            if (e != hipSuccess) {
                (void)hipGraphDestroy(graph);
                set_error(hip_msg(e, "hipGraphAddEventRecordNode"));
                return PCG_E_DEVICE;
            }
            prev = node;
        }
        return PCG_OK;
    };
    for (size_t li = 0; li < seq.size(); ++li) {
        if (add_marks(li) != PCG_OK) return PCG_E_DEVICE;
        KernelLaunch& l = seq[li];
        void* params[] = {&l.args};   // copied when the node is added
        hipKernelNodeParams np{};
        np.func = const_cast<void*>(l.func);
        np.gridDim = l.grid;
        np.blockDim = l.block;
        np.sharedMemBytes = 0;
        np.kernelParams = params;
        np.extra = nullptr;
        hipGraphNode_t node = nullptr;
        const hipError_t e = hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr,
                                                   prev ? 1 : 0, &np);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            set_error(hip_msg(e, "hipGraphAddKernelNode"));
            return PCG_E_DEVICE;
        }
        prev = node;
    }
    if (add_marks(seq.size()) != PCG_OK) return PCG_E_DEVICE;
    hipGraphExec_t exec = nullptr;
    const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    PCG_HIP(e, "hipGraphInstantiate");
    P->graphs[key] = GraphEntry{exec, now};
    *out = exec;
    return PCG_OK;
}

struct RunInfo {
    int launches = 0;
    double ms_a = 0.0, ms_b = 0.0;
    int n_a = 0, n_b = 0;
};

// Fused Krylov engine for nrhs right-hand sides of precision T.  The states
// at a.st must hold fresh_state() values with zero_start set as `zero_start`
// (x0 = 0: x is not read and the first kernel B takes r from b = a.in1).
// fixup = false: the exit correction u += alpha p is left to the caller
// (the mixed-precision update folds it in).
template <typename T>
pcg_status run_fused(pcg_problem* P, int dtype, int prec_slot, const ColArgs& a_in, int64_t nrhs,
                     bool zero_start, const pcg_solve_opts& o, char* ws, const Layout& w,
                     SolverState* host_states, RunInfo& info, hipStream_t s, bool fixup = true)
{
    // line preconditioner: z and p trade vectors after the first kernel A,
    // which then need not store p = z (the other preconditioners' kernels
    // write z into io2 throughout)
    ColArgs a = a_in;
    a.zswap = o.preconditioner == PCG_PRECOND_LINE ? 1 : 0;
    Phase bph;
    if (b_phase<T>(P, dtype, a, nrhs, o, ws, w, bph) != PCG_OK) return PCG_E_DEVICE;
    const int profile = nrhs == 1 ? o.profile : 0;   // 1: kernels A and B, 2: A only
    int K = o.graph_chunk > 0 ? o.graph_chunk : P->last_iters[prec_slot];
    if (K <= 0) K = 8;
    K = std::min(K, std::max(1, o.max_iter));
    const bool use_graph = o.graph_chunk != 0;

    // zero start: the first kernel B reads b itself; otherwise r = b - A x0
    if (!zero_start && launch<T>(Kind::InitFull, a, nrhs, s, info.launches)) return PCG_E_DEVICE;

    // profile: phase i (kernel A, or kernel B's launches up to its last main
    // kernel) is bracketed by events 2i and 2i+1
    Phase aph, aph_first, bph_first;
    if (!add_kind<T>(aph, Kind::FusedApply, a, nrhs) ||
        !add_kind<T>(aph_first, Kind::FusedApplyFirst, a, nrhs)) {
        set_error("no kernel for this shape (internal)");
        return PCG_E_DEVICE;
    }
    // kernel B's first launch: the first-launch kernel with the line
    // preconditioner (the other preconditioners' first kernels handle their
    // first launch themselves)
    if (o.preconditioner == PCG_PRECOND_LINE) {
        ColArgs af = a;
        af.x0_zero = zero_start ? 1 : 0;   // r from b (every right-hand side starts alike)
        if (!add_kind<T>(bph_first, Kind::FusedPrecFirst, af, nrhs)) {
            set_error("no kernel for this shape (internal)");
            return PCG_E_DEVICE;
        }
    } else {
        bph_first = bph;
    }
    // timings in launch order: kernel A or B, and either an event pair of
    // P->events (direct launches, each its own pair, read at the end; -1
    // once read) or the time already read (graph chunks reuse their events
    // on every replay, so each replay's are read after it)
    struct Timing {
        char is_a;
        int pair;
        float ms;
    };
    std::vector<Timing> tms;
    int pairs = 0;
    auto timed = [&](const Phase& ph, char kind_a) -> pcg_status {
        const int i = pairs++;
        if (ensure_events(P, 2 * (size_t)i + 2) != PCG_OK) return PCG_E_DEVICE;
        PCG_HIP(hipEventRecord(P->events[2 * i], s), "hipEventRecord");
        for (size_t j = 0; j < ph.k.size(); ++j) {
            PCG_HIP(issue(ph.k[j], s), "kernel launch");
            if (j == ph.last_main) PCG_HIP(hipEventRecord(P->events[2 * i + 1], s), "hipEventRecord");
        }
        info.launches += ph.mains;
        tms.push_back(Timing{kind_a, i, 0.f});
        return PCG_OK;
    };
    if (profile == 1) {
        if (timed(bph_first, 0) != PCG_OK) return PCG_E_DEVICE;
    } else if (issue_phase(bph_first, s, info.launches) != PCG_OK) {
        return PCG_E_DEVICE;
    }

    const int max_chunks = o.max_iter / K + 3;
    int chunks = 0;
    for (;;) {
        const bool first = chunks == 0;
        if (profile && !use_graph) {
            for (int i = 0; i < K; ++i) {
                if (timed((first && i == 0) ? aph_first : aph, 1) != PCG_OK) return PCG_E_DEVICE;
                if (profile == 1 ? timed(bph, 0) != PCG_OK
                                 : issue_phase(bph, s, info.launches) != PCG_OK)
                    return PCG_E_DEVICE;
            }
            if (fixup && launch<T>(Kind::Fixup, a, nrhs, s, info.launches)) return PCG_E_DEVICE;
        } else if (use_graph) {
            hipGraphExec_t exec;
            if (chunk_graph<T>(P, a, bph, nrhs, K, first, fixup, profile, &exec) != PCG_OK)
                return PCG_E_DEVICE;
            PCG_HIP(hipGraphLaunch(exec, s), "hipGraphLaunch");
            info.launches += (1 + bph.mains) * K + (fixup ? 1 : 0);
        } else {
            if (issue_chunk<T>(a, bph, nrhs, K, first, fixup, s, info.launches)) return PCG_E_DEVICE;
        }
        ++chunks;
        if (read_states(P, a.st, host_states, nrhs, s) != PCG_OK) return PCG_E_DEVICE;
        if (profile && use_graph) {   // the replay is complete: read its events
            for (int i = 0; i < K; ++i) {
                float ma = 0.f, mb = 0.f;
                PCG_HIP(hipEventElapsedTime(&ma, P->gevents[4 * i], P->gevents[4 * i + 1]),
                        "hipEventElapsedTime");
                tms.push_back(Timing{1, -1, ma});
                if (profile != 1) continue;
                PCG_HIP(hipEventElapsedTime(&mb, P->gevents[4 * i + 2], P->gevents[4 * i + 3]),
                        "hipEventElapsedTime");
                tms.push_back(Timing{0, -1, mb});
            }
        }
        bool running = false;
        for (int64_t i = 0; i < nrhs; ++i) running |= host_states[i].flag == kRunning;
        if (!running) break;
        if (chunks >= max_chunks) {
            set_error("iteration chunks exceeded the iteration limit (internal)");
            return PCG_E_DEVICE;
        }
    }
    if (profile) {
        for (Timing& t : tms)
            if (t.pair >= 0)
                PCG_HIP(hipEventElapsedTime(&t.ms, P->events[2 * t.pair], P->events[2 * t.pair + 1]),
                        "hipEventElapsedTime");
        // count the launches that did work (later ones returned at once)
        const int done_a = host_states[0].iter;
        int na = 0, nb = 0;
        for (const Timing& t : tms) {
            if (t.is_a && na < done_a) {
                info.ms_a += t.ms;
                ++na;
            } else if (!t.is_a && nb < done_a + 1) {
                info.ms_b += t.ms;
                ++nb;
            }
        }
        info.n_a = na;
        info.n_b = nb;
    }
    int maxit = 0;
    for (int64_t i = 0; i < nrhs; ++i) maxit = std::max(maxit, host_states[i].iter);
    if (maxit > 0) P->last_iters[prec_slot] = maxit;
    return PCG_OK;
}

pcg_status status_of(const SolverState& s)
{
    switch (s.flag) {
    case kConverged: return PCG_OK;
    case kMaxIter: return PCG_E_NOCONV;
    case kBreakdown: return PCG_E_BREAKDOWN;
    default: return PCG_E_NOCONV;
    }
}

ColArgs base_args(const pcg_problem* P, int dtype, char* ws, const Layout& w, int64_t bpr)
{
    ColArgs a{};
    a.g = P->geom;
    set_launch(a, P, dtype);
    a.blocks_per_rhs = bpr;
    set_tables(a, P, dtype);
    a.part = reinterpret_cast<double*>(ws + w.part);
    return a;
}

// ------------------------------------------------------------- FP64 fused --

pcg_status solve_fp64(pcg_problem* P, const double* b, double* x, char* ws, const Layout& w,
                      int64_t nrhs, const pcg_solve_opts& o, pcg_result* res, hipStream_t s)
{
    const int64_t bpr = blocks_per_rhs(P, PCG_F64);
    ColArgs a = base_args(P, PCG_F64, ws, w, bpr);
    a.in0 = x;
    a.in1 = b;
    a.io0 = x;
    a.io1 = ws + w.r;
    a.io2 = ws + w.z;
    a.io3 = ws + w.p;
    a.io4 = ws + w.q;
    a.st = reinterpret_cast<SolverState*>(ws + w.st);
    std::vector<SolverState> hs(nrhs, fresh_state(o.rtol, o.atol, o.max_iter, 1.0));
    for (auto& h : hs) h.zero_start = o.x0_zero != 0;
    if (upload_states(P, a.st, hs.data(), nrhs, s) != PCG_OK) return PCG_E_DEVICE;
    RunInfo info;
    pcg_status st =
        run_fused<double>(P, PCG_F64, 0, a, nrhs, o.x0_zero != 0, o, ws, w, hs.data(), info, s);
    if (st != PCG_OK) return st;
    if (o.true_residual) {
        ColArgs t = a;
        t.in0 = x;
        t.in1 = b;
        if (launch<double>(Kind::TrueResidual, t, nrhs, s, info.launches)) return PCG_E_DEVICE;
        if (read_states(P, a.st, hs.data(), nrhs, s) != PCG_OK) return PCG_E_DEVICE;
    }
    for (int64_t i = 0; i < nrhs; ++i) {
        pcg_result& r = res[i];
        r.status = status_of(hs[i]);
        r.iterations = hs[i].iter;
        r.outer_iterations = 0;
        r.launches = info.launches;
        r.r0_norm = hs[i].r0norm;
        r.rel_res_recursive = hs[i].r0norm > 0 ? hs[i].rnorm / hs[i].r0norm : 0.0;
        r.rel_res_true = o.true_residual ? (hs[i].r0norm > 0 ? hs[i].aux / hs[i].r0norm : 0.0) : -1.0;
        r.ms_apply_kernel = info.ms_a;
        r.ms_precond_kernel = info.ms_b;
        r.n_apply_kernel = info.n_a;
        r.n_precond_kernel = info.n_b;
    }
    return PCG_OK;
}

// ----------------------------------------------------------- FP64 unfused --

pcg_status solve_unfused(pcg_problem* P, const double* b, double* x, char* ws, const Layout& w,
                         const pcg_solve_opts& o, pcg_result* res, hipStream_t s)
{
    const int64_t bpr = blocks_per_rhs(P, PCG_F64);
    ColArgs a = base_args(P, PCG_F64, ws, w, bpr);
    SolverState* dst = reinterpret_cast<SolverState*>(ws + w.st);
    double* r = reinterpret_cast<double*>(ws + w.r);
    double* z = reinterpret_cast<double*>(ws + w.z);
    double* p = reinterpret_cast<double*>(ws + w.p);
    double* q = reinterpret_cast<double*>(ws + w.q);
    SolverState hs = fresh_state(o.rtol, o.atol, o.max_iter, 1.0);
    if (upload_states(P, dst, &hs, 1, s) != PCG_OK) return PCG_E_DEVICE;
    int launches = 0;
    BlasArgs ba{};
    ba.n = P->geom.n;
    ba.blocks = blas_blocks(P->geom.n);
    ba.st = dst;
    ba.part = a.part;
    ba.red_mode = a.red_mode;
    auto blas = [&](Blas op, const double* xx, const double* yy, double* w0) -> pcg_status {
        BlasArgs c = ba;
        c.x = xx;
        c.y = yy;
        c.w0 = w0;
        hipError_t e = launch_blas(op, c, s);
        if (e != hipSuccess) {
            set_error(hip_msg(e, "blas launch"));
            return PCG_E_DEVICE;
        }
        ++launches;
        return PCG_OK;
    };
    // start: r = b - A x, z = M^{-1} r, rho = <r,z>, p = z
    ColArgs init = a;
    init.in1 = b;
    init.io0 = x;
    init.io1 = r;
    init.io3 = p;
    init.io4 = q;
    init.st = dst;
    if (launch<double>(o.x0_zero ? Kind::InitZero : Kind::InitFull, init, 1, s, launches))
        return PCG_E_DEVICE;
    ColArgs pre = a;
    pre.in0 = r;
    pre.io0 = z;
    pre.st = dst;
    ColArgs app = a;
    app.in0 = p;
    app.io0 = q;
    app.st = dst;
    if (launch<double>(Kind::Precond, pre, 1, s, launches)) return PCG_E_DEVICE;
    if (blas(Blas::InitDot, r, z, nullptr)) return PCG_E_DEVICE;
    if (blas(Blas::CopyZP, z, nullptr, p)) return PCG_E_DEVICE;
    int K = o.graph_chunk > 0 ? o.graph_chunk : (P->last_iters[0] > 0 ? P->last_iters[0] : 8);
    K = std::min(K, std::max(1, o.max_iter));
    const int max_chunks = o.max_iter / K + 3;
    for (int chunk = 0;; ++chunk) {
        for (int i = 0; i < K; ++i) {
            if (launch<double>(Kind::Apply, app, 1, s, launches)) return PCG_E_DEVICE;  // q = A p
            if (blas(Blas::DotPQ, p, q, nullptr)) return PCG_E_DEVICE;                  // alpha
            if (blas(Blas::AxpyXP, p, nullptr, x)) return PCG_E_DEVICE;                 // x += alpha p
            if (blas(Blas::AxpyRQ, q, nullptr, r)) return PCG_E_DEVICE;                 // r -= alpha q
            if (blas(Blas::Nrm2R, r, nullptr, nullptr)) return PCG_E_DEVICE;            // ||r||, exit
            if (launch<double>(Kind::Precond, pre, 1, s, launches)) return PCG_E_DEVICE; // z = M^-1 r
            if (blas(Blas::DotRZ, r, z, nullptr)) return PCG_E_DEVICE;                  // beta
            if (blas(Blas::ScalP, nullptr, nullptr, p)) return PCG_E_DEVICE;            // p = beta p
            if (blas(Blas::AxpyPZ, z, nullptr, p)) return PCG_E_DEVICE;                 // p += z
        }
        if (read_states(P, dst, &hs, 1, s) != PCG_OK) return PCG_E_DEVICE;
        if (hs.flag != kRunning) break;
        if (chunk + 1 >= max_chunks) {
            set_error("iteration chunks exceeded the iteration limit (internal)");
            return PCG_E_DEVICE;
        }
    }
    if (hs.iter > 0) P->last_iters[0] = hs.iter;
    if (o.true_residual) {
        ColArgs t = a;
        t.in0 = x;
        t.in1 = b;
        t.st = dst;
        if (launch<double>(Kind::TrueResidual, t, 1, s, launches)) return PCG_E_DEVICE;
        if (read_states(P, dst, &hs, 1, s) != PCG_OK) return PCG_E_DEVICE;
    }
    res->status = status_of(hs);
    res->iterations = hs.iter;
    res->outer_iterations = 0;
    res->launches = launches;
    res->r0_norm = hs.r0norm;
    res->rel_res_recursive = hs.r0norm > 0 ? hs.rnorm / hs.r0norm : 0.0;
    res->rel_res_true = o.true_residual ? (hs.r0norm > 0 ? hs.aux / hs.r0norm : 0.0) : -1.0;
    return PCG_OK;
}

// -------------------------------------------------------- mixed precision --

pcg_status solve_mixed(pcg_problem* P, const double* b, double* x, char* ws, const Layout& w,
                       int64_t nrhs, const pcg_solve_opts& o, pcg_result* res, hipStream_t s)
{
    const int64_t bpr64 = blocks_per_rhs(P, PCG_F64);
    const int64_t bpr32 = blocks_per_rhs(P, PCG_F32);
    SolverState* st_in = reinterpret_cast<SolverState*>(ws + w.st);
    SolverState* st_out = reinterpret_cast<SolverState*>(ws + w.st_o);

    ColArgs outer = base_args(P, PCG_F64, ws, w, bpr64);
    outer.in0 = x;
    outer.in1 = b;
    outer.io0 = x;
    outer.out32 = ws + w.r32;   // Residual64 writes the inner right-hand side
    outer.st = st_out;

    ColArgs inner = base_args(P, PCG_F32, ws, w, bpr32);
    inner.in1 = ws + w.r32;     // b of the inner solve is r32 itself (no copy)
    inner.io0 = ws + w.u32;
    inner.io1 = ws + w.r32;
    inner.io2 = ws + w.z32;
    inner.io3 = ws + w.p32;
    inner.io4 = ws + w.q32;
    inner.st = st_in;

    ColArgs upd = outer;
    upd.out32 = ws + w.u32;     // Update64 reads the inner solution u and folds
    upd.st_in = st_in;          // in its pending exit correction alpha p, p being
    upd.in0 = o.preconditioner == PCG_PRECOND_LINE ? ws + w.z32 : ws + w.p32;   // where kernel A keeps it

    std::vector<SolverState> ho(nrhs), hi(nrhs);
    std::vector<double> r0(nrhs, 0.0), rn(nrhs, 0.0), scale(nrhs, 1.0);
    std::vector<char> done(nrhs, 0);
    std::vector<int> inner_iters(nrhs, 0), outer_steps(nrhs, 0);
    std::vector<pcg_status> stat(nrhs, PCG_E_NOCONV);
    RunInfo info;
    int launches = 0;

    for (int k = 0;; ++k) {
        for (int64_t i = 0; i < nrhs; ++i) {
            ho[i] = fresh_state(o.rtol, o.atol, 0, scale[i]);
            ho[i].flag = done[i] ? kConverged : kRunning;
        }
        if (upload_states(P, st_out, ho.data(), nrhs, s) != PCG_OK) return PCG_E_DEVICE;
        outer.x0_zero = upd.x0_zero = (k == 0 && o.x0_zero) ? 1 : 0;   // x not read yet
        if (launch<double>(Kind::Residual64, outer, nrhs, s, launches)) return PCG_E_DEVICE;
        if (read_states(P, st_out, ho.data(), nrhs, s) != PCG_OK) return PCG_E_DEVICE;
        bool all_done = true;
        for (int64_t i = 0; i < nrhs; ++i) {
            if (done[i]) continue;
            rn[i] = ho[i].rnorm;
            if (k == 0) r0[i] = rn[i];
            if (!std::isfinite(rn[i])) {
                done[i] = 1;
                stat[i] = PCG_E_BREAKDOWN;
            } else if (r0[i] == 0.0 || rn[i] / r0[i] < o.rtol || rn[i] < o.atol) {
                done[i] = 1;
                stat[i] = PCG_OK;
            } else if (k >= o.max_outer || inner_iters[i] >= o.max_iter) {
                done[i] = 1;
                stat[i] = PCG_E_NOCONV;
            }
            all_done &= done[i] != 0;
        }
        // a zero start that stops at its first residual (b = 0, ||b|| <= atol,
        // a non-finite b) has written nothing to x yet: x = x0 = 0
        if (k == 0 && o.x0_zero)
            for (int64_t i = 0; i < nrhs; ++i)
                if (done[i])
                    PCG_HIP(hipMemsetAsync(x + i * P->geom.n, 0, sizeof(double) * (size_t)P->geom.n, s),
                            "hipMemsetAsync(x = 0)");
        if (all_done) {
            PCG_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");   // the call blocks
            break;
        }
        // first step: rescale if the residual left the comfortable FP32 range
        if (k == 0) {
            bool redo = false;
            for (int64_t i = 0; i < nrhs; ++i)
                if (!done[i] && (rn[i] > 1e20 || rn[i] < 1e-20)) {
                    scale[i] = 1.0 / rn[i];
                    redo = true;
                }
            if (redo) {
                for (int64_t i = 0; i < nrhs; ++i) {
                    ho[i] = fresh_state(o.rtol, o.atol, 0, scale[i]);
                    ho[i].flag = done[i] ? kConverged : kRunning;
                }
                if (upload_states(P, st_out, ho.data(), nrhs, s) != PCG_OK) return PCG_E_DEVICE;
                if (launch<double>(Kind::Residual64, outer, nrhs, s, launches)) return PCG_E_DEVICE;
            }
        }
        // inner FP32 solve A d = r32 to inner_rtol
        for (int64_t i = 0; i < nrhs; ++i) {
            const int budget = std::max(1, o.max_iter - inner_iters[i]);
            hi[i] = fresh_state(o.inner_rtol, 0.0, budget, 1.0);
            hi[i].flag = done[i] ? kConverged : kRunning;
            hi[i].zero_start = 1;
        }
        if (upload_states(P, st_in, hi.data(), nrhs, s) != PCG_OK) return PCG_E_DEVICE;
        pcg_solve_opts io = o;
        io.max_iter = 1 << 30;
        io.profile = 0;
        pcg_status st = run_fused<float>(P, PCG_F32, 1, inner, nrhs, true, io, ws, w, hi.data(),
                                         info, s, false);
        if (st != PCG_OK) return st;
        // x += (u + alpha p) / scale
        for (int64_t i = 0; i < nrhs; ++i) {
            ho[i] = fresh_state(o.rtol, o.atol, 0, scale[i]);
            ho[i].flag = done[i] ? kConverged : kRunning;
        }
        if (upload_states(P, st_out, ho.data(), nrhs, s) != PCG_OK) return PCG_E_DEVICE;
        if (launch<double>(Kind::Update64, upd, nrhs, s, launches)) return PCG_E_DEVICE;
        for (int64_t i = 0; i < nrhs; ++i) {
            if (done[i]) continue;
            inner_iters[i] += hi[i].iter;
            outer_steps[i] += 1;
            if (hi[i].flag == kBreakdown && hi[i].iter == 0) {
                done[i] = 1;
                stat[i] = PCG_E_BREAKDOWN;
                continue;
            }
            // next residual is about ||r|| * (inner reduction); keep r32 near unit size
            const double red = hi[i].r0norm > 0 ? hi[i].rnorm / hi[i].r0norm : 1.0;
            const double est = rn[i] * std::max(red, 1e-30);
            if (std::isfinite(est) && est > 0) scale[i] = 1.0 / est;
        }
    }
    for (int64_t i = 0; i < nrhs; ++i) {
        pcg_result& r = res[i];
        r.status = stat[i];
        r.iterations = inner_iters[i];
        r.outer_iterations = outer_steps[i];
        r.launches = launches + info.launches;
        r.r0_norm = r0[i];
        r.rel_res_recursive = r0[i] > 0 ? rn[i] / r0[i] : 0.0;
        r.rel_res_true = r.rel_res_recursive;   // the outer residual is the true FP64 one
        r.ms_apply_kernel = r.ms_precond_kernel = 0.0;
        r.n_apply_kernel = r.n_precond_kernel = 0;
    }
    return PCG_OK;
}

// Time fused iterations of precision T with the problem's current tuning on
// the workspace vectors (r holds a synthetic right-hand side).  Each rep
// restarts from x0 = 0 and times the first iteration's kernels B and A, so
// the timed work never depends on convergence.  Returns ms per iteration.
template <typename T>
pcg_status time_tuning(pcg_problem* P, int dtype, int64_t nrhs, char* ws, const Layout& w,
                       void* u, hipStream_t s, float* ms_b, float* ms_a)
{
    const int64_t bpr = blocks_per_rhs(P, dtype);
    ColArgs a = base_args(P, dtype, ws, w, bpr);
    const bool f64 = dtype == PCG_F64;
    a.io0 = u;
    a.io1 = ws + (f64 ? w.r : w.r32);
    a.io2 = ws + (f64 ? w.z : w.z32);
    a.io3 = ws + (f64 ? w.p : w.p32);
    a.io4 = ws + (f64 ? w.q : w.q32);
    a.in1 = a.io1;                      // zero start in place: r keeps its data
    a.st = reinterpret_cast<SolverState*>(ws + w.st);
    const int reps = 6;
    if (ensure_events(P, 3 * reps) != PCG_OK) return PCG_E_DEVICE;
    // iter = 1: time the general kernels (alpha = beta = 0, p = q = 0 after
    // the start kernel), not the first-iteration specialisations
    std::vector<SolverState> hs(nrhs, fresh_state(0.0, 0.0, 1 << 30, 1.0));
    for (auto& h : hs) {
        h.iter = 1;
        h.r0norm = 1.0;   // the exit test divides by it
    }
    int cnt = 0;
    for (int i = -1; i < reps; ++i) {   // rep -1 warms up
        if (upload_states(P, a.st, hs.data(), nrhs, s) != PCG_OK) return PCG_E_DEVICE;
        if (launch<T>(Kind::InitZero, a, nrhs, s, cnt)) return PCG_E_DEVICE;
        if (i >= 0) PCG_HIP(hipEventRecord(P->events[3 * i], s), "hipEventRecord");
        if (launch<T>(Kind::FusedPrec, a, nrhs, s, cnt)) return PCG_E_DEVICE;
        if (i >= 0) PCG_HIP(hipEventRecord(P->events[3 * i + 1], s), "hipEventRecord");
        if (launch<T>(Kind::FusedApply, a, nrhs, s, cnt)) return PCG_E_DEVICE;
        if (i >= 0) PCG_HIP(hipEventRecord(P->events[3 * i + 2], s), "hipEventRecord");
    }
    PCG_HIP(hipEventSynchronize(P->events[3 * reps - 1]), "hipEventSynchronize");
    // the fastest repetition: other work on the device only ever slows one down
    float tb = 1e30f, ta = 1e30f;
    for (int i = 0; i < reps; ++i) {
        float b = 0.f, a2 = 0.f;
        PCG_HIP(hipEventElapsedTime(&b, P->events[3 * i], P->events[3 * i + 1]),
                "hipEventElapsedTime");
        PCG_HIP(hipEventElapsedTime(&a2, P->events[3 * i + 1], P->events[3 * i + 2]),
                "hipEventElapsedTime");
        tb = std::min(tb, b);
        ta = std::min(ta, a2);
    }
    std::vector<SolverState> out(nrhs);
    if (read_states(P, a.st, out.data(), nrhs, s) != PCG_OK) return PCG_E_DEVICE;
    for (int64_t i = 0; i < nrhs; ++i)
        if (out[i].flag != kRunning || out[i].iter != 2) {
            set_error("autotune: the synthetic first iteration did not complete (internal)");
            return PCG_E_DEVICE;
        }
    *ms_b = tb;
    *ms_a = ta;
    return PCG_OK;
}

struct DeviceBuffer {
    void* p = nullptr;
    ~DeviceBuffer()
    {
        if (p) (void)hipFree(p);
    }
};

pcg_status autotune_in(pcg_problem* P, int dtype, int64_t nrhs, char* ws, const Layout& w,
                       void* u, hipStream_t s, Tuning* best);

}  // namespace

pcg_status autotune(pcg_problem* P, int dtype, int64_t nrhs, hipStream_t s, Tuning* best)
{
    pcg_solve_opts o;
    pcg_default_opts(&o);
    o.precision = dtype == PCG_F64 ? PCG_PREC_FP64 : PCG_PREC_MIXED;
    const Layout w = plan_n(P->geom.n, o, nrhs, kMaxBlocks);   // any candidate fits
    const size_t ubytes = al256((size_t)P->geom.n * nrhs * (dtype == PCG_F64 ? 8 : 4));
    DeviceBuffer buf;
    hipError_t e = hipMalloc(&buf.p, w.total + ubytes);
    if (e != hipSuccess) {
        set_error(hip_msg(e, "pcg_autotune: hipMalloc(scratch)"));
        return PCG_E_NOMEM;
    }
    char* ws = static_cast<char*>(buf.p);
    pcg_status st = autotune_in(P, dtype, nrhs, ws, w, ws + w.total, s, best);
    (void)hipStreamSynchronize(s);
    return st;
}

namespace {

pcg_status autotune_in(pcg_problem* P, int dtype, int64_t nrhs, char* ws, const Layout& w,
                       void* u, hipStream_t s, Tuning* best)
{
    // synthetic right-hand side: every 32-bit word 0x3f800000 (1.0f; as FP64
    // words a positive number near 2^-7), so the iteration does real work
    const size_t vec_bytes = (size_t)P->geom.n * nrhs * (dtype == PCG_F64 ? 8 : 4);
    PCG_HIP(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(ws + (dtype == PCG_F64 ? w.r : w.r32)),
                              0x3f800000, vec_bytes / 4, s),
            "hipMemsetD32Async");
    const Tuning saved = P->tune[dtype];
    // per reduction mode: the three fastest launch shapes of kernel A (all
    // but the line solve) and of kernel B, timed with the same shape for both
    struct Pick {
        float ms = 1e30f;
        Shape sh;
        int64_t cap = kDefaultCap;
    };
    constexpr int kTop = 3;
    Pick top_a[2][kTop], top_b[2][kTop];
    auto keep = [](Pick (&top)[kTop], const Pick& p) {
        for (int i = 0; i < kTop; ++i)
            if (p.ms < top[i].ms) {
                for (int j = kTop - 1; j > i; --j) top[j] = top[j - 1];
                top[i] = p;
                return;
            }
    };
    auto time_pair = [&](const Tuning& t, float* ms_b, float* ms_a) -> pcg_status {
        P->tune[dtype] = t;
        return dtype == PCG_F64 ? time_tuning<double>(P, dtype, nrhs, ws, w, u, s, ms_b, ms_a)
                                : time_tuning<float>(P, dtype, nrhs, ws, w, u, s, ms_b, ms_a);
    };
    const int nz = P->geom.nz;
    for (int L = 1; L <= kWave; L <<= 1) {
        Shape sh;
        sh.L = L;
        if (!shape_supported(nz, sh)) continue;
        sh.M = 1;
        while (sh.M * L < nz) sh.M <<= 1;
        if (sh.M * L >= 2 * nz && L > 1 && sh.M > 1) continue;   // lanes idle: skip
        for (int64_t total = 512; total <= kMaxBlocks; total <<= 1) {
            const int64_t cap = std::max<int64_t>(1, std::min<int64_t>(kMaxBlocks, total / nrhs));
            if (column_blocks(P->geom, sh) < cap && total > 512) continue;  // no change
            for (int mode = 0; mode < 2; ++mode) {
                Tuning t;
                t.shape = sh;
                t.block_cap = cap;
                t.red_mode = mode;
                t.shape_b = sh;
                t.block_cap_b = cap;
                float ms_b = 0.f, ms_a = 0.f;
                const pcg_status st = time_pair(t, &ms_b, &ms_a);
                if (st != PCG_OK) {
                    P->tune[dtype] = saved;
                    return st;
                }
                keep(top_a[mode], Pick{ms_a, sh, cap});
                keep(top_b[mode], Pick{ms_b, sh, cap});
            }
        }
    }
    // the shapes of A and B interact (how B stores z changes A's reads of
    // it), so the final choice times the combinations of the leaders
    Tuning best_t;
    float best_ms = 1e30f;
    for (int mode = 0; mode < 2; ++mode)
        for (int i = 0; i < kTop; ++i)
            for (int j = 0; j < kTop; ++j) {
                if (top_a[mode][i].ms >= 1e30f || top_b[mode][j].ms >= 1e30f) continue;
                Tuning t;
                t.shape = top_a[mode][i].sh;
                t.block_cap = top_a[mode][i].cap;
                t.shape_b = top_b[mode][j].sh;
                t.block_cap_b = top_b[mode][j].cap;
                t.red_mode = mode;
                float ms_b = 0.f, ms_a = 0.f;
                const pcg_status st = time_pair(t, &ms_b, &ms_a);
                if (st != PCG_OK) {
                    P->tune[dtype] = saved;
                    return st;
                }
                if (ms_a + ms_b < best_ms) {
                    best_ms = ms_a + ms_b;
                    best_t = t;
                }
            }
    P->tune[dtype] = best_t;
    if (best) *best = best_t;
    return PCG_OK;
}

}  // namespace

// Multigrid preconditioner alone: bytes of scratch (the fine level's t and
// r, t, z of every coarse level) and one V-cycle z = B r.
size_t mg_bytes(const pcg_problem* P, int dtype, int levels_req)
{
    const size_t elem = dtype == PCG_F64 ? sizeof(double) : sizeof(float);
    Layout w;
    plan_mg(P, mg_levels_used(P, levels_req), 1, elem, w);
    return w.total;
}

pcg_status mg_precond(pcg_problem* P, int dtype, const void* r, void* z, int levels_req,
                      void* workspace, size_t ws_bytes, hipStream_t s)
{
    TuneScope ts(P, 1);
    const size_t elem = dtype == PCG_F64 ? sizeof(double) : sizeof(float);
    Layout w;
    plan_mg(P, mg_levels_used(P, levels_req), 1, elem, w);
    if (ws_bytes < w.total) {
        std::ostringstream m;
        m << "pcg_mg_precond: workspace of " << ws_bytes << " bytes is smaller than the "
          << w.total << " needed";
        set_error(m.str());
        return PCG_E_NOMEM;
    }
    char* ws = static_cast<char*>(workspace);
    ColArgs a{};
    a.g = P->geom;
    set_launch(a, P, dtype);
    set_tables(a, P, dtype);
    MgVecs v{};
    v.r[0] = const_cast<void*>(r);
    v.t[0] = ws + w.mg_t[0];
    v.z[0] = z;
    for (int l = 1; l < w.mg_levels; ++l) {
        v.r[l] = ws + w.mg_r[l];
        v.t[l] = ws + w.mg_t[l];
        v.z[l] = ws + w.mg_z[l];
    }
    Phase ph;
    const bool ok = dtype == PCG_F64 ? mg_phase<double>(P, dtype, a, 1, w.mg_levels, v, false, ph)
                                     : mg_phase<float>(P, dtype, a, 1, w.mg_levels, v, false, ph);
    if (!ok) {
        set_error("no kernel for this shape (internal)");
        return PCG_E_DEVICE;
    }
    int count = 0;
    return issue_phase(ph, s, count);
}

bool rbgs_supported(const pcg_problem* P)
{
    return !((P->geom.per_x && P->geom.nx % 2) || (P->geom.per_y && P->geom.ny % 2));
}

// Block Gauss-Seidel preconditioner alone: z = M^{-1} r.
pcg_status rbgs_precond(pcg_problem* P, int dtype, const void* r, void* z, hipStream_t s)
{
    TuneScope ts(P, 1);
    ColArgs a{};
    a.g = P->geom;
    set_launch(a, P, dtype);
    set_tables(a, P, dtype);
    a.in0 = r;
    a.io2 = z;
    Phase ph;
    const bool ok =
        dtype == PCG_F64
            ? add_kind<double>(ph, Kind::RbFirst, a, 1) && add_kind<double>(ph, Kind::RbBlack, a, 1) &&
                  add_kind<double>(ph, Kind::RbRed, a, 1)
            : add_kind<float>(ph, Kind::RbFirst, a, 1) && add_kind<float>(ph, Kind::RbBlack, a, 1) &&
                  add_kind<float>(ph, Kind::RbRed, a, 1);
    if (!ok) {
        set_error("no kernel for this shape (internal)");
        return PCG_E_DEVICE;
    }
    int count = 0;
    return issue_phase(ph, s, count);
}

// Workspace of one served request, enough for any tuning of its shape (and
// the coarse levels of the multigrid preconditioner when it is chosen).
size_t request_bytes(const pcg_problem_desc& d, const pcg_solve_opts& o0)
{
    pcg_solve_opts o = o0;
    o.preconditioner = resolve_precond(d, d.dx, o0);
    const int64_t n = (int64_t)d.nx * d.ny * d.nz;
    size_t total = plan_n(n, o, 1, kMaxBlocks).total;
    if (o.preconditioner == PCG_PRECOND_MG) {
        const size_t elem = o.precision == PCG_PREC_MIXED ? sizeof(float) : sizeof(double);
        int64_t nx = d.nx, ny = d.ny;
        int levels = 1;
        total += al256(elem * (size_t)n);
        while (nx % 2 == 0 && ny % 2 == 0 && nx / 2 >= kMgMinCells && ny / 2 >= kMgMinCells &&
               (o.mg_levels <= 0 || levels < o.mg_levels)) {
            nx /= 2;
            ny /= 2;
            ++levels;
            total += 3 * al256(elem * (size_t)(nx * ny * d.nz));
        }
    }
    return total;
}

size_t workspace_bytes(const pcg_problem* Pc, const pcg_solve_opts& o, int64_t nrhs)
{
    pcg_problem* P = const_cast<pcg_problem*>(Pc);
    TuneScope ts(P, nrhs);
    return plan(P, o, nrhs).total;
}

pcg_status solve(pcg_problem* P, const double* b, double* x, void* workspace, size_t ws_bytes,
                 const pcg_solve_opts& o0, int64_t nrhs, pcg_result* res, hipStream_t s)
{
    TuneScope ts(P, nrhs);
    const pcg_solve_opts o = resolved_opts(P, o0);
    if (o.preconditioner == PCG_PRECOND_RBGS && !rbgs_supported(P)) {
        set_error("block Gauss-Seidel: red-black ordering needs an even size in periodic "
                  "directions");
        return PCG_E_INVALID;
    }
    const Layout w = plan(P, o, nrhs);
    if (ws_bytes < w.total) {
        std::ostringstream m;
        m << "workspace of " << ws_bytes << " bytes is smaller than the " << w.total << " needed";
        set_error(m.str());
        return PCG_E_NOMEM;
    }
    char* ws = static_cast<char*>(workspace);
    const auto t0 = std::chrono::steady_clock::now();
    pcg_status st;
    if (o.precision == PCG_PREC_MIXED) st = solve_mixed(P, b, x, ws, w, nrhs, o, res, s);
    else if (o.fused) st = solve_fp64(P, b, x, ws, w, nrhs, o, res, s);
    else st = solve_unfused(P, b, x, ws, w, o, res, s);
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (st != PCG_OK) return st;
    pcg_status worst = PCG_OK;
    for (int64_t i = 0; i < nrhs; ++i) {
        res[i].elapsed_ms = ms;
        res[i].preconditioner = o.preconditioner;
        if (res[i].status == PCG_E_BREAKDOWN) worst = PCG_E_BREAKDOWN;
        else if (res[i].status == PCG_E_NOCONV && worst == PCG_OK) worst = PCG_E_NOCONV;
    }
    return worst;
}

}  // namespace pcg
