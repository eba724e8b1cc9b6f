"""The C oracle and the library's host-only C++ (descriptor validation and
column tables, the tuning-cache parser, the serving arena) built with
AddressSanitizer and UndefinedBehaviorSanitizer (gcc/g++, no GPU code) and
driven over small, edge-case and malformed inputs: any out-of-bounds access,
use after free, leak or undefined operation aborts the driver."""
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
