"""The C oracle and the library's host-only C++ (descriptor validation and
column tables, the tuning-cache parser, the serving arena) built with
AddressSanitizer and UndefinedBehaviorSanitizer (gcc/g++, no GPU code) and
driven over small, edge-case and malformed inputs: any out-of-bounds access,
use after free, leak or undefined operation aborts the driver.

The server's request queue (csrc/server.cpp, per-request worker mode) built
host-only with ThreadSanitizer, and again with AddressSanitizer and
UndefinedBehaviorSanitizer, against stand-ins for the HIP runtime calls it
makes (host memory, synchronous copies) and a mock solve: several client
threads submit, cancel, poll and wait while a monitor thread queries the
statistics; any data race, deadlock report or memory error aborts the
driver, and the results and counters are checked."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1302_7193_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")

ORACLE_DRIVER = r'''
#include <assert.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
long orc_assemble(int, int, int, double, double, double, double, double, double, int, int,
                  int64_t *, int32_t *, double *);
long orc_assemble_geom(int, int, int, const double *, const double *, double, double, double,
                       double, int, int, int64_t *, int32_t *, double *);
void orc_line_blocks(long, int, const int64_t *, const int32_t *, const double *, double *,
                     double *, double *);
void orc_line_solve(long, int, const double *, const double *, const double *, const double *,
                    double *, double *);
int orc_pcg(long, int, const int64_t *, const int32_t *, const double *, const double *,
            const double *, const double *, const double *, double *, double, double, int,
            double *, double *);
double orc_residual_norm(long, const int64_t *, const int32_t *, const double *, const double *,
                         const double *);
double orc_row_apply(int, int, int, double, double, double, double, double, double, int, int,
                     int, int, int, const double *);
void orc_csr_matvec(long, const int64_t *, const int32_t *, const double *, const double *,
                    double *);

static void run(int nx, int ny, int nz, int px, int py, double kh, int stretched) {
    const long n = (long)nx * ny * nz;
    int64_t *rp = malloc(sizeof(int64_t) * (n + 1));
    int32_t *col = malloc(sizeof(int32_t) * 7 * n);
    double *val = malloc(sizeof(double) * 7 * n), *b = malloc(sizeof(double) * n);
    double *x = calloc(n, sizeof(double)), *y = malloc(sizeof(double) * n);
    double *lo = malloc(sizeof(double) * n), *di = malloc(sizeof(double) * n);
    double *up = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
    double *work = malloc(sizeof(double) * 2 * nz), out[4];
    long nnz;
    if (stretched) {
        double *xw = malloc(sizeof(double) * nx), *yw = malloc(sizeof(double) * ny);
        for (int i = 0; i < nx; ++i) xw[i] = (1.0 + 0.5 * (i % 3)) / nx;
        for (int j = 0; j < ny; ++j) yw[j] = (1.0 + 0.25 * (j % 2)) / ny;
        nnz = orc_assemble_geom(nx, ny, nz, xw, yw, 1.0, 1.05, kh, 40.0, px, py, rp, col, val);
        free(xw);
        free(yw);
    } else {
        nnz = orc_assemble(nx, ny, nz, 1.0 / nx, 1.0 / ny, 1.0, 1.05, kh, 40.0, px, py, rp, col,
                           val);
    }
    assert(nnz > 0 && nnz <= 7 * n && rp[n] == nnz);
    for (long i = 0; i < n; ++i) b[i] = sin(0.37 * i) + 0.1;
    orc_csr_matvec(n, rp, col, val, b, y);
    for (int k = 0; k < nz; ++k) {     /* the matrix-free row formula on column 0 */
        const double r = orc_row_apply(nx, ny, nz, 1.0 / nx, 1.0 / ny, 1.0, 1.05, kh, 40.0, px,
                                       py, 0, 0, k, b);
        if (!stretched) assert(fabs(r - y[k]) <= 1e-12 * (fabs(r) + 1.0));
    }
    orc_line_blocks(n, nz, rp, col, val, lo, di, up);
    orc_line_solve(n, nz, lo, di, up, b, z, work);
    const int st = orc_pcg(n, nz, rp, col, val, lo, di, up, b, x, 1e-10, 0.0, 500, out, NULL);
    assert(st == 0);
    assert(orc_residual_norm(n, rp, col, val, b, x) <= 1e-9 * orc_residual_norm(n, rp, col, val,
                                                                                b, z) + 1e-300
           || orc_residual_norm(n, rp, col, val, b, x) < 1e-8);
    free(rp); free(col); free(val); free(b); free(x); free(y);
    free(lo); free(di); free(up); free(z); free(work);
}

int main(void) {
    run(5, 4, 7, 0, 0, 1.0, 0);
    run(3, 3, 1, 1, 1, 1.0, 0);      /* one level; periodic at the minimum size */
    run(1, 1, 40, 0, 0, 1.0, 0);     /* one column */
    run(6, 5, 9, 1, 0, 0.0, 0);      /* no horizontal coupling */
    run(7, 4, 12, 0, 1, 1.0, 1);     /* stretched */
    puts("oracle ok");
    return 0;
}
'''

HOST_DRIVER = r'''
#include <cassert>
#include <cstdio>
#include <fstream>
#include <random>
#include <string>
#include <vector>
#include "arena.h"
#include "problem.h"

namespace pcg {
std::string validate(const pcg_problem_desc& d);
void build_tables(const pcg_problem_desc& d, Geom& g, std::vector<double>& vert,
                  std::vector<double>& lu);
std::string stretched_geometry(const pcg_problem_desc& d, const double* xw, const double* yw,
                               std::vector<double>& hgeo);
void set_error(const std::string&) {}
}

static pcg_problem_desc desc(int nx, int ny, int nz, double q, int per) {
    pcg_problem_desc d{};
    d.nx = nx; d.ny = ny; d.nz = nz; d.dx = 1.0 / nx; d.dy = 1.0 / ny; d.height = 1.0;
    d.grading = q; d.k_h = 1.0; d.k_v = 1e3; d.bc_x = per; d.bc_y = per;
    return d;
}

int main(int argc, char** argv) {
    // descriptors: valid ones build finite tables, invalid ones are rejected
    const int nzs[] = {1, 2, 7, 64, 128, 1000, 1024};
    for (int nz : nzs) {
        pcg_problem_desc d = desc(5, 3, nz, 1.05, 0);
        assert(pcg::validate(d).empty());
        pcg::Geom g{};
        std::vector<double> vert, lu;
        pcg::build_tables(d, g, vert, lu);
        for (double v : vert) assert(std::isfinite(v));
        for (double v : lu) assert(std::isfinite(v));
        std::vector<double> w(5, 0.2), hy(3, 1.0 / 3), hgeo;
        assert(pcg::stretched_geometry(d, w.data(), hy.data(), hgeo).empty());
        assert(hgeo.size() == 3 * (5 + 3));
    }
    assert(!pcg::validate(desc(0, 3, 4, 1.05, 0)).empty());
    assert(!pcg::validate(desc(4, 3, 2000, 1.05, 0)).empty());
    assert(!pcg::validate(desc(2, 5, 4, 1.05, 1)).empty());   // periodic needs 3 cells
    assert(!pcg::validate(desc(4, 4, 4, -1.0, 0)).empty());
    {
        pcg_problem_desc d = desc(4, 3, 4, 1.05, 0);
        std::vector<double> bad(4, 0.25), hy(3, 1.0 / 3), hgeo;
        bad[2] = -1.0;
        assert(!pcg::stretched_geometry(d, bad.data(), hy.data(), hgeo).empty());
    }

    // tuning cache: malformed, truncated and out-of-range lines are skipped
    const std::string path = argv[1];
    {
        std::ofstream f(path);
        f << "# comment\n\n"
          << "gfx950 uniform 64 64 32 0 1 8 512 1 8 512\n"
          << "gfx950 uniform 64 64 32 1 1 8 512 1\n"            // short form
          << "gfx950 uniform 64 64\n"                           // truncated
          << "gfx950 weird 64 64 32 0 1 8 512 1\n"              // bad geometry
          << "gfx950 uniform 64 64 32 0 3 3 512 1\n"            // L not a power of two
          << "gfx950 uniform 64 64 32 0 5 8 99999999 1\n"       // cap too large
          << "gfx950 uniform 64 64 32 0 7 8 512 5\n"            // bad reduction mode
          << "gfx950 uniform 64 64 2048 0 1 64 512 1\n"         // n_z beyond any shape
          << std::string(5000, 'x') << "\n"                    // overlong garbage
          << "gfx950 stretched 8 8 8 0 1 1 1 0 1 1 # trailing comment\n";
    }
    assert(pcg_tuning_cache_load(path.c_str()) == PCG_OK);
    assert(pcg_tuning_cache_load((path + ".missing").c_str()) == PCG_E_INVALID);
    pcg_problem P;
    P.arch = "gfx950";
    P.geom.nx = 64; P.geom.ny = 64; P.geom.nz = 32;
    pcg::Tuning t;
    assert(pcg::tuning_lookup(&P, 0, 1, &t) && t.shape.L == 8 && t.block_cap == 512);
    assert(pcg::tuning_lookup(&P, 1, 1, &t) && t.shape_b.L == 8);
    for (int nrhs : {3, 5, 7}) assert(!pcg::tuning_lookup(&P, 0, nrhs, &t));
    pcg::tuning_store(&P, 0, 2, t);
    assert(pcg_tuning_cache_save((path + ".out").c_str()) == PCG_OK);
    assert(pcg_tuning_cache_load((path + ".out").c_str()) == PCG_OK);
    assert(pcg::tuning_lookup(&P, 0, 2, &t));

    // arena: random allocations and releases stay consistent
    pcg::Arena a(1 << 20);
    std::mt19937 rng(7);
    std::vector<size_t> live;
    for (int it = 0; it < 20000; ++it) {
        size_t off;
        if (live.empty() || rng() % 3) {
            if (a.alloc(1 + rng() % 50000, &off)) live.push_back(off);
        } else {
            const size_t k = rng() % live.size();
            assert(a.release(live[k]));
            live.erase(live.begin() + k);
        }
    }
    for (size_t off : live) assert(a.release(off));
    assert(a.in_use() == 0 && a.free_blocks() == 1);
    std::puts("host ok");
    return 0;
}
'''


SERVER_HIP_STUBS = r'''
/* Host stand-ins for the HIP runtime calls of the server: device and pinned
   memory are host memory, copies are synchronous, streams and events are
   tokens.  C linkage and plain types (hipStream_t and hipEvent_t are
   pointers, hipError_t 0 is success). */
#include <stdlib.h>
#include <string.h>
static void* al(size_t n) { return aligned_alloc(256, (n + 255) & ~(size_t)255); }
int hipSetDevice(int d) { (void)d; return 0; }
int hipGetDevice(int* d) { *d = 0; return 0; }
int hipStreamCreateWithFlags(void** s, unsigned f) { (void)f; *s = malloc(16); return *s ? 0 : 2; }
int hipStreamDestroy(void* s) { free(s); return 0; }
int hipStreamSynchronize(void* s) { (void)s; return 0; }
int hipStreamWaitEvent(void* s, void* e, unsigned f) { (void)s; (void)e; (void)f; return 0; }
int hipEventCreateWithFlags(void** e, unsigned f) { (void)f; *e = malloc(16); return *e ? 0 : 2; }
int hipEventDestroy(void* e) { free(e); return 0; }
int hipEventRecord(void* e, void* s) { (void)e; (void)s; return 0; }
int hipMalloc(void** p, size_t n) { *p = al(n); return *p ? 0 : 2; }
int hipFree(void* p) { free(p); return 0; }
int hipHostMalloc(void** p, size_t n, unsigned f) { (void)f; *p = al(n); return *p ? 0 : 2; }
int hipHostFree(void* p) { free(p); return 0; }
int hipMemcpyAsync(void* d, const void* s, size_t n, int k, void* st)
{ (void)k; (void)st; memcpy(d, s, n); return 0; }
int hipMemsetAsync(void* d, int v, size_t n, void* st) { (void)st; memset(d, v, n); return 0; }
'''

SERVER_LIB_STUBS = r'''
// Stand-ins for the library functions the server calls: a mock solve that
// reads b and writes x = b / 2 after a short random delay, problem objects
// carrying only their size, the error message kept per thread.
#include <chrono>
#include <cstring>
#include <random>
#include <string>
#include <thread>
#include "multi.h"
#include "problem.h"

namespace pcg {
static thread_local std::string g_err;
void set_error(const std::string& m) { g_err = m; }
std::string validate(const pcg_problem_desc& d)
{
    return d.nx > 0 && d.ny > 0 && d.nz > 0 ? std::string() : std::string("sizes");
}
size_t request_bytes(const pcg_problem_desc& d, const pcg_solve_opts&)
{
    return 32 * (size_t)d.nx * d.ny * d.nz + 4096;
}
int resolve_precond(const pcg_problem_desc&, double, const pcg_solve_opts& o)
{
    return o.preconditioner;
}
int64_t column_blocks(const Geom&, const Shape&) { return 1; }
hipError_t multi_launch(MultiOp, const MultiTable*, int64_t, int, hipStream_t)
{
    return hipErrorInvalidValue;   // batched mode is not driven here
}
pcg_status solve(pcg_problem* P, const double* b, double* x, void* ws, size_t ws_bytes,
                 const pcg_solve_opts& o, int64_t nrhs, pcg_result* res, hipStream_t)
{
    if (!P || !b || !x || !ws || nrhs != 1 || ws_bytes < request_bytes(P->desc, o)) {
        set_error("mock solve: bad arguments");
        return PCG_E_INVALID;
    }
    static thread_local std::mt19937 rng(std::hash<std::thread::id>()(std::this_thread::get_id()));
    std::this_thread::sleep_for(std::chrono::microseconds(50 + rng() % 400));
    std::memset(ws, 0, ws_bytes);
    for (int64_t i = 0; i < P->geom.n; ++i) x[i] = 0.5 * b[i];
    std::memset(res, 0, sizeof(*res));
    res->status = PCG_OK;
    res->iterations = 1;
    return PCG_OK;
}
}  // namespace pcg

extern "C" {
pcg_status pcg_problem_create(const pcg_problem_desc* d, pcg_problem** out)
{
    pcg_problem* P = new pcg_problem();
    P->desc = *d;
    P->geom.nx = d->nx; P->geom.ny = d->ny; P->geom.nz = d->nz;
    P->geom.n = (int64_t)d->nx * d->ny * d->nz;
    *out = P;
    return PCG_OK;
}
void pcg_problem_destroy(pcg_problem* P) { delete P; }
void pcg_default_opts(pcg_solve_opts* o)
{
    std::memset(o, 0, sizeof(*o));
    o->rtol = 1e-8;
    o->max_iter = 100;
    o->fused = 1;
    o->graph_chunk = -1;
}
size_t pcg_last_error(char* buf, size_t n)
{
    const std::string& e = pcg::g_err;
    if (buf && n) {
        std::strncpy(buf, e.c_str(), n - 1);
        buf[n - 1] = 0;
    }
    return e.size();
}
}
'''

SERVER_DRIVER = r'''
#include <atomic>
#include <cassert>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>
#include "pcg.h"

int main()
{
    const size_t arena_bytes = size_t(16) << 20;
    void* arena = aligned_alloc(256, arena_bytes);
    pcg_server_opts so{};
    so.hbm_budget_bytes = size_t(3) << 20;   // admission waits for memory as well as workers
    so.max_active = 4;
    so.batched = 0;
    pcg_server* S = nullptr;
    assert(pcg_server_create(&so, arena, arena_bytes, &S) == PCG_OK);
    constexpr int kUsers = 6, kPerUser = 30;
    std::atomic<bool> stop{false};
    std::atomic<int> ok{0}, cancelled{0};
    std::thread monitor([&] {
        pcg_server_stats st;
        while (!stop.load()) {
            assert(pcg_server_query(S, &st) == PCG_OK);
            assert(st.active <= so.max_active && st.bytes_in_use <= so.hbm_budget_bytes);
            std::this_thread::yield();
        }
    });
    std::vector<std::thread> users;
    for (int u = 0; u < kUsers; ++u)
        users.emplace_back([&, u] {
            std::mt19937 rng(u + 1);
            for (int i = 0; i < kPerUser; ++i) {
                pcg_problem_desc d{};
                d.nx = 4 + rng() % 29;
                d.ny = 4 + rng() % 29;
                d.nz = 8 << (rng() % 3);
                d.dx = 1.0 / d.nx; d.dy = 1.0 / d.ny; d.height = 1.0;
                d.grading = 1.05; d.k_h = 1.0; d.k_v = 1e3;
                const size_t n = (size_t)d.nx * d.ny * d.nz;
                std::vector<double> b(n), x(n, -1.0);
                for (size_t k = 0; k < n; ++k) b[k] = double(k % 97) + u;
                uint64_t t = 0;
                assert(pcg_submit(S, &d, nullptr, b.data(), x.data(), &t) == PCG_OK);
                pcg_result res;
                pcg_status st;
                if (i % 5 == 4 && pcg_cancel(S, t) == PCG_OK) {
                    assert(pcg_wait(S, t, &res) == PCG_E_CANCELLED);
                    ++cancelled;
                    continue;
                }
                if (i % 2) {
                    while ((st = pcg_poll(S, t, &res)) == PCG_E_AGAIN) std::this_thread::yield();
                } else {
                    st = pcg_wait(S, t, &res);
                }
                assert(st == PCG_OK && res.iterations == 1);
                for (size_t k = 0; k < n; ++k) assert(x[k] == 0.5 * b[k]);
                ++ok;
            }
        });
    for (auto& t : users) t.join();
    stop = true;
    monitor.join();
    pcg_server_stats st;
    assert(pcg_server_query(S, &st) == PCG_OK);
    assert(st.submitted == (uint64_t)(kUsers * kPerUser));
    assert(st.completed + st.cancelled == st.submitted);
    assert(st.completed == (uint64_t)ok.load() && st.cancelled == (uint64_t)cancelled.load());
    assert(st.active == 0 && st.queued == 0 && st.bytes_in_use == 0);
    assert(st.peak_active >= 2 && st.peak_active <= so.max_active);
    assert(st.peak_bytes_in_use <= so.hbm_budget_bytes);
    pcg_server_destroy(S);
    free(arena);
    std::printf("server ok: %d completed, %d cancelled, peak %d active\n", ok.load(),
                cancelled.load(), st.peak_active);
    return 0;
}
'''


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (cmd, r.stdout[-3000:], r.stderr[-3000:])
    return r


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    drv = tmp_path / "oracle_driver.c"
    drv.write_text(ORACLE_DRIVER)
    exe = tmp_path / "oracle_san"
    _run(["gcc", "-std=c99"] + SAN + [str(drv), os.path.join(ROOT, "oracle", "pcg_oracle.c"),
                                      "-o", str(exe), "-lm"])
    r = _run([str(exe)], env=ENV, timeout=300)
    assert "oracle ok" in r.stdout


def test_host_code_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    drv = tmp_path / "host_driver.cpp"
    drv.write_text(HOST_DRIVER)
    exe = tmp_path / "host_san"
    _run(["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
          "-I" + os.path.join(ROOT, "include"), "-I" + CSRC] + SAN +
         [str(drv), os.path.join(CSRC, "problem.cpp"), os.path.join(CSRC, "tuning_cache.cpp"),
          "-o", str(exe), "-ldl"])
    r = _run([str(exe), str(tmp_path / "cache.txt")], env=ENV, timeout=300)
    assert "host ok" in r.stdout


def _server_build(tmp_path, san):
    files = {"hip_stubs.c": SERVER_HIP_STUBS, "lib_stubs.cpp": SERVER_LIB_STUBS,
             "driver.cpp": SERVER_DRIVER}
    for name, text in files.items():
        (tmp_path / name).write_text(text)
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    _run(["gcc", "-std=c11", "-c"] + san + [str(tmp_path / "hip_stubs.c"), "-o",
                                           str(tmp_path / "hip_stubs.o")])
    exe = tmp_path / "server_san"
    _run(["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"] + inc + san +
         [os.path.join(CSRC, "server.cpp"), str(tmp_path / "lib_stubs.cpp"),
          str(tmp_path / "driver.cpp"), str(tmp_path / "hip_stubs.o"), "-o", str(exe),
          "-lpthread"])
    return exe


def test_server_queue_under_thread_sanitizer(tmp_path):
    exe = _server_build(tmp_path, ["-fsanitize=thread", "-g", "-O1"])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:second_deadlock_stack=1")
    r = _run([str(exe)], env=env, timeout=300)
    assert "server ok" in r.stdout and "ThreadSanitizer" not in r.stderr


def test_server_queue_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = _server_build(tmp_path, SAN)
    r = _run([str(exe)], env=ENV, timeout=300)
    assert "server ok" in r.stdout
