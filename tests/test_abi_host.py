"""Host-only checks of the C ABI library: it loads, exports every entry point
declared in include/pcg.h, its structs have the layout the binding assumes,
and the pure-host entry points validate their arguments.  No kernel is
launched here."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pcg.h")
LIB = os.path.join(ROOT, "paper_1302_7193_amd", "libpcg.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pcg_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_entry_point(lib):
    names = declared_functions()
    assert len(names) >= 13
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (pcg_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        getattr(lib, n)


def test_struct_layouts_match_header(tmp_path):
    import paper_1302_7193_amd as pcg
    prog = tmp_path / "sizes.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "pcg.h"\n'
                    'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n",'
                    ' sizeof(pcg_problem_desc), sizeof(pcg_solve_opts), sizeof(pcg_result),'
                    ' offsetof(pcg_result, ms_apply_kernel), offsetof(pcg_solve_opts, inner_rtol),'
                    ' sizeof(pcg_tuning), sizeof(pcg_server_opts), sizeof(pcg_server_stats),'
                    ' offsetof(pcg_server_stats, peak_active));'
                    'return 0;}\n')
    exe = tmp_path / "sizes"
    subprocess.check_call(["gcc", "-I" + os.path.join(ROOT, "include"), str(prog), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(pcg.pcg_problem_desc), ctypes.sizeof(pcg.pcg_solve_opts),
            ctypes.sizeof(pcg.pcg_result), pcg.pcg_result.ms_apply_kernel.offset,
            pcg.pcg_solve_opts.inner_rtol.offset, ctypes.sizeof(pcg.pcg_tuning),
            ctypes.sizeof(pcg.pcg_server_opts), ctypes.sizeof(pcg.pcg_server_stats),
            pcg.pcg_server_stats.peak_active.offset]
    assert got == want


def test_default_opts():
    import paper_1302_7193_amd as pcg
    o = pcg.pcg_default_opts()
    assert (o.rtol, o.atol, o.max_iter, o.fused, o.graph_chunk) == (1e-8, 0.0, 10000, 1, -1)
    assert o.precision == pcg.PCG_PREC_FP64 and o.inner_rtol == 3e-5 and o.max_outer == 20


@pytest.mark.parametrize("nx,nz,g2,kv", [(64, 32, 1e4, 4e4), (512, 128, 1e5, 1.6e6),
                                         (1024, 128, 1e4, 6.4e5), (256, 64, 1e3, 1.6e4)])
def test_desc_from_ratio_closed_form(nx, nz, g2, kv):
    import paper_1302_7193_amd as pcg
    d = pcg.pcg_desc_from_ratio(nx, nx, nz, 1.05, g2, pcg.PCG_BC_PERIODIC)
    assert abs(d.k_v - kv) <= 1e-12 * kv
    assert (d.dx, d.dy, d.height, d.k_h, d.grading) == (1.0 / nx, 1.0 / nx, 1.0, 1.0, 1.05)
    assert d.bc_x == d.bc_y == pcg.PCG_BC_PERIODIC


@pytest.mark.parametrize("args,msg", [
    ((2, 8, 8, 1.05, 1e3, 1), "periodic"),          # periodic needs >= 3 cells
    ((8, 8, 2048, 1.05, 1e3, 0), "exceeds"),        # n_z above the column limit
    ((0, 8, 8, 1.05, 1e3, 0), "sizes"),
    ((8, 8, 8, 1.05, -1.0, 0), "gamma2"),
])
def test_desc_validation_errors(args, msg):
    import paper_1302_7193_amd as pcg
    with pytest.raises(pcg.PCGError) as e:
        pcg.pcg_desc_from_ratio(*args)
    assert e.value.status == pcg.PCG_E_INVALID
    assert msg in str(e.value)


def test_workspace_and_csr_sizes_are_host_computable():
    # pcg_csr_bytes / pcg_workspace_bytes need no device; they need a problem
    # handle, which needs a device, so only the NULL-handle contract is
    # checked here.
    import paper_1302_7193_amd as pcg
    assert pcg._lib.pcg_csr_bytes(None, 0) == 0
    assert pcg._lib.pcg_workspace_bytes(None, None, 1) == 0
    assert pcg._lib.pcg_apply(None, 0, None, None, None) == pcg.PCG_E_INVALID
    assert "NULL" in pcg.pcg_last_error()


def test_tuning_cache_file_round_trip(lib, tmp_path):
    """The tuning cache parses its text format (skipping comments and
    malformed or unsupported entries) and writes back what it holds."""
    src = tmp_path / "in.txt"
    src.write_text("# comment line\n"
                   "gfx950 uniform 97 89 61 0 1 16 2048 1   # trailing comment\n"
                   "gfx950 stretched 97 89 61 1 64 32 65536 0 8 1024\n"
                   "gfx950 stretched 97 89 61 0 64 32 65536 0 8\n"       # prec cap missing
                   "gfx950 uniform 97 89 61 0 1 48 2048 1\n"      # L not a power of two
                   "gfx950 uniform 97 89 61 0 1 16 0 1\n"         # block cap below 1
                   "gfx950 uniform 97 89 61 2 1 16 2048 1\n"      # unknown dtype
                   "gfx950 curved 97 89 61 0 1 16 2048 1\n"       # unknown geometry
                   "gfx950 uniform 97 89\n")                      # truncated
    lib.pcg_tuning_cache_load.argtypes = [ctypes.c_char_p]
    lib.pcg_tuning_cache_save.argtypes = [ctypes.c_char_p]
    assert lib.pcg_tuning_cache_load(str(src).encode()) == 0
    assert lib.pcg_tuning_cache_load(str(tmp_path / "missing.txt").encode()) != 0
    out = tmp_path / "out.txt"
    assert lib.pcg_tuning_cache_save(str(out).encode()) == 0
    rows = [ln.split() for ln in out.read_text().splitlines() if ln and not ln.startswith("#")]
    mine = sorted(r for r in rows if r[2:5] == ["97", "89", "61"])
    assert mine == [["gfx950", "stretched", "97", "89", "61", "1", "64", "32", "65536", "0", "8",
                     "1024"],
                    ["gfx950", "uniform", "97", "89", "61", "0", "1", "16", "2048", "1", "16",
                     "2048"]]


def test_stretched_create_rejects_bad_widths_before_touching_a_device(lib):
    import paper_1302_7193_amd as pcg
    d = pcg.pcg_desc_from_ratio(4, 3, 8, 1.05, 1e3, pcg.PCG_BC_DIRICHLET)
    h = ctypes.c_void_p()
    dp = ctypes.POINTER(ctypes.c_double)
    f = lib.pcg_problem_create_stretched
    f.argtypes = [ctypes.POINTER(pcg.pcg_problem_desc), dp, dp, ctypes.POINTER(ctypes.c_void_p)]
    good_x, good_y = (ctypes.c_double * 4)(0.25, 0.25, 0.25, 0.25), (ctypes.c_double * 3)(1, 2, 3)
    for xs, ys in (((0.25, 0.0, 0.25, 0.5), (1, 2, 3)), ((0.25, 0.25, 0.25, 0.25), (1, -2, 3)),
                   ((0.25, float("nan"), 0.25, 0.5), (1, 2, 3))):
        xa, ya = (ctypes.c_double * 4)(*xs), (ctypes.c_double * 3)(*ys)
        assert f(ctypes.byref(d), xa, ya, ctypes.byref(h)) == pcg.PCG_E_INVALID
        assert not h.value
    assert f(ctypes.byref(d), None, good_y, ctypes.byref(h)) == pcg.PCG_E_INVALID
    assert f(ctypes.byref(d), good_x, None, ctypes.byref(h)) == pcg.PCG_E_INVALID


def test_stream_probe_rejects_bad_arguments_before_touching_a_device(lib):
    import paper_1302_7193_amd as pcg
    f = pcg._lib.pcg_stream_probe
    buf = (ctypes.c_void_p * 7)(*[0x10000 * (k + 1) for k in range(7)])
    for nr, nw, nbytes, nt, blocks in ((0, 1, 1024, 1, 0), (5, 1, 1024, 1, 0), (1, 0, 1024, 1, 0),
                                       (1, 4, 1024, 1, 0), (1, 1, 0, 1, 0), (1, 1, 1000, 1, 0),
                                       (1, 1, 1024, 4, 0), (1, 1, 1024, -1, 0),
                                       (1, 1, 1024, 1, -1)):
        assert f(nr, nw, buf, nbytes, nt, blocks, None) == pcg.PCG_E_INVALID, (nr, nw, nbytes)
    assert f(1, 1, None, 1024, 1, 0, None) == pcg.PCG_E_INVALID
    bad = (ctypes.c_void_p * 2)(0x10000, 0x20008)            # misaligned
    assert f(1, 1, bad, 1024, 1, 0, None) == pcg.PCG_E_INVALID
    overlap = (ctypes.c_void_p * 2)(0x10000, 0x10200)        # written overlaps read
    assert f(1, 1, overlap, 1024, 1, 0, None) == pcg.PCG_E_INVALID
    assert "overlaps" in pcg.pcg_last_error()
