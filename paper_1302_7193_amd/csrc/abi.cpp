// extern "C" entry points of libpcg (declared in include/pcg.h).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <initializer_list>
#include <new>
#include <sstream>
#include <string>

#include "problem.h"

namespace pcg {

std::string validate(const pcg_problem_desc& d);
std::string stretched_geometry(const pcg_problem_desc& d, const double* xw, const double* yw,
                               std::vector<double>& hgeo);
void build_tables(const pcg_problem_desc& d, Geom& g, std::vector<double>& vert,
                  std::vector<double>& lu);
size_t workspace_bytes(const pcg_problem* P, const pcg_solve_opts& o, int64_t nrhs);
size_t mg_bytes(const pcg_problem* P, int dtype, int levels_req);
pcg_status rbgs_precond(pcg_problem* P, int dtype, const void* r, void* z, hipStream_t s);
bool rbgs_supported(const pcg_problem* P);
pcg_status mg_precond(pcg_problem* P, int dtype, const void* r, void* z, int levels_req,
                      void* workspace, size_t ws_bytes, hipStream_t s);
int64_t blocks_per_rhs(const pcg_problem* P, int dtype);
pcg_status autotune(pcg_problem* P, int dtype, int64_t nrhs, hipStream_t s, Tuning* best);
pcg_status solve_noalloc(pcg_problem* P, const double* b, double* x, const pcg_solve_opts& o,
                         pcg_result* res, hipStream_t s);
pcg_status solve(pcg_problem* P, const double* b, double* x, void* workspace, size_t ws_bytes,
                 const pcg_solve_opts& o, int64_t nrhs, pcg_result* res, hipStream_t s);

namespace {
thread_local std::string g_last_error;

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

std::string hip_msg(hipError_t e, const char* what)
{
    std::ostringstream m;
    m << what << ": " << hipGetErrorName(e) << " (" << hipGetErrorString(e) << ")";
    return m.str();
}

// Runs f with the problem's device current and restores the caller's.
template <typename F>
pcg_status on_device(int dev, F&& f)
{
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) cur = -1;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) {
        set_error("hipSetDevice failed");
        return PCG_E_DEVICE;
    }
    pcg_status s;
    try {
        s = f();
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        s = PCG_E_NOMEM;
    } catch (...) {
        set_error("unexpected exception inside libpcg");
        s = PCG_E_DEVICE;
    }
    if (cur >= 0 && cur != dev) (void)hipSetDevice(cur);
    return s;
}

bool valid_dtype(int32_t d) { return d == PCG_F64 || d == PCG_F32; }

// The column kernels move 16-byte vectors: every device pointer crossing the
// ABI must be 16-byte aligned.
bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

pcg_status check_aligned(std::initializer_list<const void*> ptrs, const char* where)
{
    for (const void* p : ptrs)
        if (!aligned16(p)) {
            set_error(std::string(where) + ": device pointers must be 16-byte aligned");
            return PCG_E_INVALID;
        }
    return PCG_OK;
}

// Two byte ranges [a, a + na) and [b, b + nb) share a byte.
bool overlap(const void* a, size_t na, const void* b, size_t nb)
{
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return na > 0 && nb > 0 && x < y + nb && y < x + na;
}

// Rejects an output range that shares bytes with an input range; with
// exact_ok an output that is exactly the input (same start, in-place
// kernels) is allowed.
pcg_status check_disjoint(const void* in, const void* out, size_t bytes, bool exact_ok,
                          const char* what)
{
    if (exact_ok && in == out) return PCG_OK;
    if (overlap(in, bytes, out, bytes)) {
        set_error(what);
        return PCG_E_INVALID;
    }
    return PCG_OK;
}

size_t elem_bytes(int32_t dtype) { return dtype == PCG_F64 ? sizeof(double) : sizeof(float); }

pcg_status check_opts(const pcg_solve_opts& o)
{
    if (!(o.rtol >= 0.0) || !(o.atol >= 0.0) || !std::isfinite(o.rtol) || !std::isfinite(o.atol)) {
        set_error("rtol and atol must be finite and >= 0");
        return PCG_E_INVALID;
    }
    if (o.max_iter < 1) {
        set_error("max_iter must be >= 1");
        return PCG_E_INVALID;
    }
    if (o.precision != PCG_PREC_FP64 && o.precision != PCG_PREC_MIXED) {
        set_error("precision must be PCG_PREC_FP64 or PCG_PREC_MIXED");
        return PCG_E_INVALID;
    }
    if (o.precision == PCG_PREC_MIXED &&
        (!(o.inner_rtol > 0.0 && o.inner_rtol < 1.0) || o.max_outer < 1)) {
        set_error("mixed precision needs 0 < inner_rtol < 1 and max_outer >= 1");
        return PCG_E_INVALID;
    }
    if (o.precision == PCG_PREC_MIXED && !o.fused) {
        set_error("mixed precision runs the fused iteration only");
        return PCG_E_INVALID;
    }
    if (o.graph_chunk < -1) {
        set_error("graph_chunk must be -1, 0 or positive");
        return PCG_E_INVALID;
    }
    if (o.profile < 0 || o.profile > 2) {
        set_error("profile must be 0, 1 or 2");
        return PCG_E_INVALID;
    }
    if (o.preconditioner < PCG_PRECOND_LINE || o.preconditioner > PCG_PRECOND_AUTO ||
        o.mg_levels < 0) {
        set_error("preconditioner must be PCG_PRECOND_LINE, _MG, _RBGS or _AUTO, mg_levels >= 0");
        return PCG_E_INVALID;
    }
    if (o.preconditioner != PCG_PRECOND_LINE && o.preconditioner != PCG_PRECOND_AUTO && !o.fused) {
        set_error("the multigrid and block Gauss-Seidel preconditioners run in the fused "
                  "iteration only");
        return PCG_E_INVALID;
    }
    return PCG_OK;
}

}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

}  // namespace pcg

using namespace pcg;

extern "C" {

void pcg_default_opts(pcg_solve_opts* o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->rtol = 1e-8;
    o->atol = 0.0;
    o->max_iter = 10000;
    o->precision = PCG_PREC_FP64;
    o->inner_rtol = 3e-5;
    o->max_outer = 20;
    o->fused = 1;
    o->graph_chunk = -1;
    o->profile = 0;
    o->true_residual = 0;
    o->x0_zero = 0;
}

pcg_status pcg_desc_from_ratio(int32_t nx, int32_t ny, int32_t nz, double grading, double gamma2,
                               int32_t bc, pcg_problem_desc* out)
{
    if (!out) {
        set_error("out is NULL");
        return PCG_E_INVALID;
    }
    if (nx < 1 || ny < 1 || nz < 1 || !(gamma2 > 0.0) || !std::isfinite(gamma2)) {
        set_error("pcg_desc_from_ratio: sizes must be >= 1 and gamma2 > 0");
        return PCG_E_INVALID;
    }
    pcg_problem_desc d{};
    d.nx = nx;
    d.ny = ny;
    d.nz = nz;
    d.dx = 1.0 / nx;
    d.dy = 1.0 / ny;
    d.height = 1.0;
    d.grading = grading;
    d.k_h = 1.0;
    const double dzbar = d.height / nz;
    d.k_v = gamma2 * d.k_h * dzbar * dzbar / (d.dx * d.dx);
    d.bc_x = d.bc_y = bc;
    const std::string err = validate(d);
    if (!err.empty()) {
        set_error(err);
        return PCG_E_INVALID;
    }
    *out = d;
    return PCG_OK;
}

// Coarse multigrid levels: 2 x 2 horizontal cells merged per level (widths
// of neighbouring cells summed) while n_x and n_y are even and both halves
// keep kMgMinCells cells; every level's column LU factors (uniform) or
// per-index geometry (stretched), in one device allocation.
static pcg_status build_mg_levels(pcg_problem* P, const double* xw, const double* yw)
{
    pcg_problem_desc d = P->desc;
    std::vector<double> wx, wy;
    if (xw) {
        wx.assign(xw, xw + d.nx);
        wy.assign(yw, yw + d.ny);
    }
    std::vector<double> vert;
    while (d.nx % 2 == 0 && d.ny % 2 == 0 && d.nx / 2 >= kMgMinCells && d.ny / 2 >= kMgMinCells) {
        d.nx /= 2;
        d.ny /= 2;
        d.dx *= 2.0;
        d.dy *= 2.0;
        MgLevel m;
        build_tables(d, m.g, vert, m.lu64);
        if (xw) {
            for (int i = 0; i < d.nx; ++i) wx[i] = wx[2 * i] + wx[2 * i + 1];
            for (int j = 0; j < d.ny; ++j) wy[j] = wy[2 * j] + wy[2 * j + 1];
            wx.resize(d.nx);
            wy.resize(d.ny);
            const std::string err = stretched_geometry(d, wx.data(), wy.data(), m.hgeo);
            if (!err.empty()) {
                set_error(err);
                return PCG_E_INVALID;
            }
        }
        P->mg.push_back(std::move(m));
    }
    if (P->mg.empty()) return PCG_OK;
    size_t total = 0;
    for (const MgLevel& m : P->mg)
        total += al256(8 * m.lu64.size()) + al256(4 * m.lu64.size()) + al256(8 * m.hgeo.size());
    hipError_t e = hipMalloc(&P->mg_tables, total);
    if (e != hipSuccess) {
        set_error(hip_msg(e, "hipMalloc(multigrid tables)"));
        return PCG_E_NOMEM;
    }
    std::vector<char> host(total, 0);
    size_t off = 0;
    char* base = static_cast<char*>(P->mg_tables);
    for (MgLevel& m : P->mg) {
        const size_t nl = m.lu64.size(), ng = m.hgeo.size();
        std::memcpy(host.data() + off, m.lu64.data(), 8 * nl);
        m.d_lu64 = reinterpret_cast<const double*>(base + off);
        off += al256(8 * nl);
        float* l32 = reinterpret_cast<float*>(host.data() + off);
        for (size_t i = 0; i < nl; ++i) l32[i] = (float)m.lu64[i];
        m.d_lu32 = reinterpret_cast<const float*>(base + off);
        off += al256(4 * nl);
        if (ng) {
            std::memcpy(host.data() + off, m.hgeo.data(), 8 * ng);
            m.d_hgeo = reinterpret_cast<const double*>(base + off);
        }
        off += al256(8 * ng);
    }
    e = hipMemcpy(P->mg_tables, host.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        set_error(hip_msg(e, "hipMemcpy(multigrid tables)"));
        return PCG_E_DEVICE;
    }
    return PCG_OK;
}

static pcg_status create_problem(const pcg_problem_desc* desc, const double* xw, const double* yw,
                                 pcg_problem** out)
{
    if (!desc || !out) {
        set_error("desc/out is NULL");
        return PCG_E_INVALID;
    }
    *out = nullptr;
    std::string err = validate(*desc);
    std::vector<double> hgeo;
    if (err.empty() && xw) err = stretched_geometry(*desc, xw, yw, hgeo);
    if (!err.empty()) {
        set_error(err);
        return PCG_E_INVALID;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        set_error("no HIP device");
        return PCG_E_DEVICE;
    }
    pcg_problem* P = new (std::nothrow) pcg_problem();
    if (!P) {
        set_error("host allocation failed");
        return PCG_E_NOMEM;
    }
    P->desc = *desc;
    P->device = dev;
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            std::string a = prop.gcnArchName;
            P->arch = a.substr(0, a.find(':'));
        }
        if (P->arch.empty()) P->arch = "unknown";
    }
    build_tables(*desc, P->geom, P->vert64, P->lu64);
    P->hgeo = std::move(hgeo);
    for (int d = 0; d < 2; ++d) {
        P->tune[d].shape = default_shape(desc->nz, d);
        P->tune[d].block_cap = kDefaultCap;
        P->tune[d].red_mode = 1;
        P->tune[d].shape_b = P->tune[d].shape;
        P->tune[d].block_cap_b = kDefaultCap;
    }
    const size_t nv = P->vert64.size(), nl = P->lu64.size(), ng = P->hgeo.size();
    const size_t b64v = al256(8 * nv), b64l = al256(8 * nl), b32v = al256(4 * nv),
                 b32l = al256(4 * nl), bg = al256(8 * ng);
    const size_t total = b64v + b64l + b32v + b32l + bg;
    hipError_t e = hipMalloc(&P->dev_tables, total);
    if (e != hipSuccess) {
        set_error(hip_msg(e, "hipMalloc(tables)"));
        delete P;
        return PCG_E_NOMEM;
    }
    std::vector<char> host(total, 0);
    std::memcpy(host.data(), P->vert64.data(), 8 * nv);
    std::memcpy(host.data() + b64v, P->lu64.data(), 8 * nl);
    float* v32 = reinterpret_cast<float*>(host.data() + b64v + b64l);
    float* l32 = reinterpret_cast<float*>(host.data() + b64v + b64l + b32v);
    for (size_t i = 0; i < nv; ++i) v32[i] = (float)P->vert64[i];
    for (size_t i = 0; i < nl; ++i) l32[i] = (float)P->lu64[i];
    if (ng) std::memcpy(host.data() + b64v + b64l + b32v + b32l, P->hgeo.data(), 8 * ng);
    e = hipMemcpy(P->dev_tables, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        set_error(hip_msg(e, "hipMemcpy(tables)"));
        (void)hipFree(P->dev_tables);
        delete P;
        return PCG_E_DEVICE;
    }
    char* base = static_cast<char*>(P->dev_tables);
    P->d_vert64 = reinterpret_cast<const double*>(base);
    P->d_lu64 = reinterpret_cast<const double*>(base + b64v);
    P->d_vert32 = reinterpret_cast<const float*>(base + b64v + b64l);
    P->d_lu32 = reinterpret_cast<const float*>(base + b64v + b64l + b32v);
    if (ng) P->d_hgeo = reinterpret_cast<const double*>(base + b64v + b64l + b32v + b32l);
    const pcg_status mst = build_mg_levels(P, xw, yw);
    if (mst != PCG_OK) {
        pcg_problem_destroy(P);
        return mst;
    }
    // pinned staging of one solver state: single-right-hand-side solves then
    // allocate nothing per call
    e = hipHostMalloc((void**)&P->pinned_states, sizeof(SolverState), 0);
    if (e != hipSuccess) {
        set_error(hip_msg(e, "hipHostMalloc(solver state)"));
        pcg_problem_destroy(P);
        return PCG_E_NOMEM;
    }
    P->pinned_cap = 1;
    *out = P;
    return PCG_OK;
}

pcg_status pcg_problem_create(const pcg_problem_desc* desc, pcg_problem** out)
{
    return create_problem(desc, nullptr, nullptr, out);
}

pcg_status pcg_problem_create_stretched(const pcg_problem_desc* desc, const double* x_widths,
                                        const double* y_widths, pcg_problem** out)
{
    if (!x_widths || !y_widths) {
        if (out) *out = nullptr;
        set_error("pcg_problem_create_stretched: width arrays must not be NULL");
        return PCG_E_INVALID;
    }
    return create_problem(desc, x_widths, y_widths, out);
}

void pcg_problem_destroy(pcg_problem* P)
{
    if (!P) return;
    int cur = -1;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(P->device);
    for (auto& kv : P->graphs) (void)hipGraphExecDestroy(kv.second.exec);
    for (hipEvent_t e : P->events) (void)hipEventDestroy(e);
    for (hipEvent_t e : P->gevents) (void)hipEventDestroy(e);
    if (P->pinned_states) (void)hipHostFree(P->pinned_states);
    if (P->dev_tables) (void)hipFree(P->dev_tables);
    if (P->mg_tables) (void)hipFree(P->mg_tables);
    if (cur >= 0) (void)hipSetDevice(cur);
    delete P;
}

size_t pcg_workspace_bytes(const pcg_problem* P, const pcg_solve_opts* opts, int32_t nrhs)
{
    if (!P || nrhs < 1) return 0;
    pcg_solve_opts o;
    if (opts) o = *opts;
    else pcg_default_opts(&o);
    return workspace_bytes(P, o, nrhs);
}

pcg_status pcg_apply(pcg_problem* P, int32_t dtype, const void* x, void* y, void* stream)
{
    if (!P || !x || !y || !valid_dtype(dtype)) {
        set_error("pcg_apply: NULL argument or bad dtype");
        return PCG_E_INVALID;
    }
    if (check_disjoint(x, y, (size_t)P->geom.n * elem_bytes(dtype), false,
                       "pcg_apply: x and y must not overlap") != PCG_OK)
        return PCG_E_INVALID;
    if (check_aligned({x, y}, "pcg_apply") != PCG_OK) return PCG_E_INVALID;
    return on_device(P->device, [&]() -> pcg_status {
        TuneScope ts(P, 1);
        ColArgs a{};
        a.g = P->geom;
        set_launch(a, P, dtype);
        set_tables(a, P, dtype);
        a.in0 = x;
        a.io0 = y;
        hipStream_t s = static_cast<hipStream_t>(stream);
        hipError_t e = dtype == PCG_F64 ? launch_column<double>(Kind::Apply, a, 1, s)
                                        : launch_column<float>(Kind::Apply, a, 1, s);
        if (e != hipSuccess) {
            set_error(hip_msg(e, "pcg_apply launch"));
            return PCG_E_DEVICE;
        }
        return PCG_OK;
    });
}

pcg_status pcg_precond(pcg_problem* P, int32_t dtype, const void* r, void* z, void* stream)
{
    if (!P || !r || !z || !valid_dtype(dtype)) {
        set_error("pcg_precond: NULL argument or bad dtype");
        return PCG_E_INVALID;
    }
    if (check_disjoint(r, z, (size_t)P->geom.n * elem_bytes(dtype), true,
                       "pcg_precond: r and z must be the same vector or not overlap") != PCG_OK)
        return PCG_E_INVALID;
    if (check_aligned({r, z}, "pcg_precond") != PCG_OK) return PCG_E_INVALID;
    return on_device(P->device, [&]() -> pcg_status {
        TuneScope ts(P, 1);
        ColArgs a{};
        a.g = P->geom;
        set_launch(a, P, dtype);
        set_tables(a, P, dtype);
        a.in0 = r;
        a.io0 = z;
        hipStream_t s = static_cast<hipStream_t>(stream);
        hipError_t e = dtype == PCG_F64 ? launch_column<double>(Kind::Precond, a, 1, s)
                                        : launch_column<float>(Kind::Precond, a, 1, s);
        if (e != hipSuccess) {
            set_error(hip_msg(e, "pcg_precond launch"));
            return PCG_E_DEVICE;
        }
        return PCG_OK;
    });
}

int32_t pcg_mg_levels(const pcg_problem* P) { return P ? 1 + (int32_t)P->mg.size() : 0; }

pcg_status pcg_rbgs_precond(pcg_problem* P, int32_t dtype, const void* r, void* z, void* stream)
{
    if (!P || !r || !z || !valid_dtype(dtype)) {
        set_error("pcg_rbgs_precond: NULL argument or bad dtype");
        return PCG_E_INVALID;
    }
    if (check_disjoint(r, z, (size_t)P->geom.n * elem_bytes(dtype), false,
                       "pcg_rbgs_precond: r and z must not overlap") != PCG_OK)
        return PCG_E_INVALID;
    if (!rbgs_supported(P)) {
        set_error("pcg_rbgs_precond: red-black ordering needs an even size in periodic directions");
        return PCG_E_INVALID;
    }
    if (check_aligned({r, z}, "pcg_rbgs_precond") != PCG_OK) return PCG_E_INVALID;
    return on_device(P->device, [&]() -> pcg_status {
        return rbgs_precond(P, dtype, r, z, static_cast<hipStream_t>(stream));
    });
}

size_t pcg_mg_bytes(const pcg_problem* P, int32_t dtype, int32_t mg_levels)
{
    if (!P || !valid_dtype(dtype) || mg_levels < 0) return 0;
    return mg_bytes(P, dtype, mg_levels);
}

pcg_status pcg_mg_precond(pcg_problem* P, int32_t dtype, const void* r, void* z,
                          int32_t mg_levels, void* workspace, size_t workspace_bytes,
                          void* stream)
{
    if (!P || !r || !z || !workspace || !valid_dtype(dtype) || mg_levels < 0) {
        set_error("pcg_mg_precond: NULL argument, bad dtype or mg_levels < 0");
        return PCG_E_INVALID;
    }
    {
        const size_t vb = (size_t)P->geom.n * elem_bytes(dtype);
        if (check_disjoint(r, z, vb, false, "pcg_mg_precond: r and z must not overlap") != PCG_OK)
            return PCG_E_INVALID;
        if (overlap(workspace, workspace_bytes, r, vb) || overlap(workspace, workspace_bytes, z, vb)) {
            set_error("pcg_mg_precond: the workspace must not overlap r or z");
            return PCG_E_INVALID;
        }
    }
    if (check_aligned({r, z, workspace}, "pcg_mg_precond") != PCG_OK) return PCG_E_INVALID;
    return on_device(P->device, [&]() -> pcg_status {
        return mg_precond(P, dtype, r, z, mg_levels, workspace, workspace_bytes,
                          static_cast<hipStream_t>(stream));
    });
}

static pcg_status solve_common(pcg_problem* P, int32_t nrhs, const double* b, double* x,
                               void* workspace, size_t workspace_bytes,
                               const pcg_solve_opts* opts, pcg_result* results, void* stream)
{
    if (!P || !b || !x || !workspace || !results || nrhs < 1) {
        set_error("pcg_solve: NULL argument or nrhs < 1");
        return PCG_E_INVALID;
    }
    pcg_solve_opts o;
    if (opts) o = *opts;
    else pcg_default_opts(&o);
    pcg_status c = check_opts(o);
    if (c != PCG_OK) return c;
    if (nrhs > 1 && !o.fused) {
        set_error("pcg_solve_batched runs the fused iteration only");
        return PCG_E_INVALID;
    }
    {
        const size_t vb = (size_t)P->geom.n * (size_t)nrhs * sizeof(double);
        if (overlap(b, vb, x, vb)) {
            set_error("pcg_solve: b and x must not overlap");
            return PCG_E_INVALID;
        }
        if (overlap(workspace, workspace_bytes, b, vb) || overlap(workspace, workspace_bytes, x, vb)) {
            set_error("pcg_solve: the workspace must not overlap b or x");
            return PCG_E_INVALID;
        }
    }
    if (check_aligned({b, x, workspace}, "pcg_solve") != PCG_OK) return PCG_E_INVALID;
    for (int32_t i = 0; i < nrhs; ++i) std::memset(&results[i], 0, sizeof(pcg_result));
    return on_device(P->device, [&]() -> pcg_status {
        return solve(P, b, x, workspace, workspace_bytes, o, nrhs, results,
                     static_cast<hipStream_t>(stream));
    });
}

pcg_status pcg_solve(pcg_problem* P, const double* b, double* x, void* workspace,
                     size_t workspace_bytes, const pcg_solve_opts* opts, pcg_result* result,
                     void* stream)
{
    return solve_common(P, 1, b, x, workspace, workspace_bytes, opts, result, stream);
}

pcg_status pcg_solve_noalloc(pcg_problem* P, const double* b, double* x,
                             const pcg_solve_opts* opts, pcg_result* result, void* stream)
{
    if (!P || !b || !x || !result) {
        set_error("pcg_solve_noalloc: NULL argument");
        return PCG_E_INVALID;
    }
    pcg_solve_opts o;
    if (opts) o = *opts;
    else pcg_default_opts(&o);
    pcg_status c = check_opts(o);
    if (c != PCG_OK) return c;
    if (overlap(b, (size_t)P->geom.n * sizeof(double), x, (size_t)P->geom.n * sizeof(double))) {
        set_error("pcg_solve_noalloc: b and x must not overlap");
        return PCG_E_INVALID;
    }
    if (check_aligned({b, x}, "pcg_solve_noalloc") != PCG_OK) return PCG_E_INVALID;
    std::memset(result, 0, sizeof(pcg_result));
    return on_device(P->device, [&]() -> pcg_status {
        return solve_noalloc(P, b, x, o, result, static_cast<hipStream_t>(stream));
    });
}

pcg_status pcg_solve_batched(pcg_problem* P, int32_t nrhs, const double* b, double* x,
                             void* workspace, size_t workspace_bytes, const pcg_solve_opts* opts,
                             pcg_result* results, void* stream)
{
    return solve_common(P, nrhs, b, x, workspace, workspace_bytes, opts, results, stream);
}

pcg_status pcg_get_tuning(const pcg_problem* P, int32_t dtype, pcg_tuning* out)
{
    if (!P || !out || !valid_dtype(dtype)) {
        set_error("pcg_get_tuning: NULL argument or bad dtype");
        return PCG_E_INVALID;
    }
    const Tuning t = effective_tuning(P, dtype, 1);
    out->lanes_per_column = t.shape.L;
    out->block_cap = (int32_t)t.block_cap;
    out->reduction = t.red_mode;
    out->lanes_per_column_prec = t.shape_b.L;
    out->block_cap_prec = (int32_t)t.block_cap_b;
    return PCG_OK;
}

pcg_status pcg_set_tuning(pcg_problem* P, int32_t dtype, const pcg_tuning* t)
{
    if (!P || !t || !valid_dtype(dtype)) {
        set_error("pcg_set_tuning: NULL argument or bad dtype");
        return PCG_E_INVALID;
    }
    Shape sh, sh_b;
    sh.L = t->lanes_per_column;
    sh_b.L = t->lanes_per_column_prec;
    if (!shape_supported(P->geom.nz, sh) || !shape_supported(P->geom.nz, sh_b)) {
        set_error("pcg_set_tuning: lanes_per_column and lanes_per_column_prec must be powers "
                  "of two in [1, 64] with 16 * lanes >= n_z");
        return PCG_E_INVALID;
    }
    if (t->block_cap < 1 || t->block_cap > kMaxBlocks || t->block_cap_prec < 1 ||
        t->block_cap_prec > kMaxBlocks || (t->reduction != 0 && t->reduction != 1)) {
        set_error("pcg_set_tuning: block caps must be in [1, 65536] and reduction 0 or 1");
        return PCG_E_INVALID;
    }
    sh.M = 1;
    while (sh.M * sh.L < P->geom.nz) sh.M <<= 1;
    sh_b.M = 1;
    while (sh_b.M * sh_b.L < P->geom.nz) sh_b.M <<= 1;
    P->tune[dtype].shape = sh;
    P->tune[dtype].block_cap = t->block_cap;
    P->tune[dtype].red_mode = t->reduction;
    P->tune[dtype].shape_b = sh_b;
    P->tune[dtype].block_cap_b = t->block_cap_prec;
    P->tune_explicit[dtype] = true;
    return PCG_OK;
}

pcg_status pcg_autotune(pcg_problem* P, int32_t dtype, int32_t nrhs, void* stream,
                        pcg_tuning* best)
{
    if (!P || !valid_dtype(dtype) || nrhs < 1) {
        set_error("pcg_autotune: NULL problem, bad dtype or nrhs < 1");
        return PCG_E_INVALID;
    }
    Tuning t;
    pcg_status st = on_device(P->device, [&]() -> pcg_status {
        return autotune(P, dtype, nrhs, static_cast<hipStream_t>(stream), &t);
    });
    if (st != PCG_OK) return st;
    P->tune[dtype] = t;
    P->tune_explicit[dtype] = true;
    tuning_store(P, dtype, nrhs, t);
    if (best) {
        best->lanes_per_column = t.shape.L;
        best->block_cap = (int32_t)t.block_cap;
        best->reduction = t.red_mode;
        best->lanes_per_column_prec = t.shape_b.L;
        best->block_cap_prec = (int32_t)t.block_cap_b;
    }
    return PCG_OK;
}

size_t pcg_csr_bytes(const pcg_problem* P, int32_t dtype)
{
    if (!P || !valid_dtype(dtype)) return 0;
    return csr_bytes(P->geom, dtype);
}

pcg_status pcg_csr_build(pcg_problem* P, int32_t dtype, void* buf, size_t bytes, void* stream)
{
    if (!P || !buf || !valid_dtype(dtype)) {
        set_error("pcg_csr_build: NULL argument or bad dtype");
        return PCG_E_INVALID;
    }
    if (check_aligned({buf}, "pcg_csr_build") != PCG_OK) return PCG_E_INVALID;
    if (bytes < csr_bytes(P->geom, dtype)) {
        set_error("pcg_csr_build: buffer smaller than pcg_csr_bytes()");
        return PCG_E_NOMEM;
    }
    return on_device(P->device, [&]() -> pcg_status {
        hipError_t e = csr_build(P->geom, P->d_vert64, P->d_hgeo, dtype, buf,
                                 static_cast<hipStream_t>(stream));
        if (e != hipSuccess) {
            set_error(hip_msg(e, "pcg_csr_build launch"));
            return PCG_E_DEVICE;
        }
        return PCG_OK;
    });
}

pcg_status pcg_csr_apply(pcg_problem* P, int32_t dtype, const void* buf, const void* x, void* y,
                         void* stream)
{
    if (!P || !buf || !x || !y || !valid_dtype(dtype)) {
        set_error("pcg_csr_apply: NULL argument or bad dtype");
        return PCG_E_INVALID;
    }
    {
        const size_t vb = (size_t)P->geom.n * elem_bytes(dtype);
        if (check_disjoint(x, y, vb, false, "pcg_csr_apply: x and y must not overlap") != PCG_OK)
            return PCG_E_INVALID;
        if (overlap(buf, csr_bytes(P->geom, dtype), y, vb)) {
            set_error("pcg_csr_apply: y must not overlap the CSR buffer");
            return PCG_E_INVALID;
        }
    }
    if (check_aligned({buf, x, y}, "pcg_csr_apply") != PCG_OK) return PCG_E_INVALID;
    return on_device(P->device, [&]() -> pcg_status {
        hipError_t e = csr_apply(P->geom, dtype, buf, x, y, static_cast<hipStream_t>(stream));
        if (e != hipSuccess) {
            set_error(hip_msg(e, "pcg_csr_apply launch"));
            return PCG_E_DEVICE;
        }
        return PCG_OK;
    });
}

pcg_status pcg_stream_probe(int32_t n_read, int32_t n_write, void* const* vectors, size_t bytes,
                            int32_t nontemporal, int64_t blocks, void* stream)
{
    if (n_read < 1 || n_read > 4 || n_write < 1 || n_write > 3 || !vectors || bytes == 0 ||
        bytes % 16 != 0 || nontemporal < 0 || nontemporal > 3 || blocks < 0) {
        set_error("pcg_stream_probe: 1..4 read and 1..3 written vectors, bytes a positive "
                  "multiple of 16, nontemporal 0..3, blocks >= 0");
        return PCG_E_INVALID;
    }
    const int nv = n_read + n_write;
    for (int i = 0; i < nv; ++i) {
        const char* v = static_cast<const char*>(vectors[i]);
        if (!v || !aligned16(v)) {
            set_error("pcg_stream_probe: vectors must be non-NULL and 16-byte aligned");
            return PCG_E_INVALID;
        }
        for (int k = 0; k < i; ++k) {
            const char* u = static_cast<const char*>(vectors[k]);
            if (v < u + bytes && u < v + bytes && (i >= n_read || k >= n_read)) {
                set_error("pcg_stream_probe: a written vector overlaps another vector");
                return PCG_E_INVALID;
            }
        }
    }
    const hipError_t e = stream_probe(n_read, n_write, vectors, bytes, nontemporal,
                                      blocks > 0 ? blocks : kDefaultCap,
                                      static_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
        set_error(hip_msg(e, "pcg_stream_probe launch"));
        return PCG_E_DEVICE;
    }
    return PCG_OK;
}

size_t pcg_last_error(char* buf, size_t n)
{
    const std::string& m = g_last_error;
    if (buf && n > 0) {
        const size_t c = m.size() < n - 1 ? m.size() : n - 1;
        std::memcpy(buf, m.data(), c);
        buf[c] = '\0';
    }
    return m.size();
}

}  // extern "C"
