"""GPU parity of libpcg against the CPU oracle, through the C ABI.

Tolerances (FP64 unit roundoff u = 1.1e-16, FP32 u = 6.0e-8):
* operator: elementwise |y_gpu - y_ref| <= 64 u (|A||x|)_i -- a 7-term sum
  evaluated in a different order from coefficients computed by a different
  formula (each a few roundings away from the oracle's);
* line preconditioner: per column, the backward error
  ||M_c z_c - r_c|| / (||M_c|| ||z_c||) <= 64 u (256 u in FP32), which does
  not depend on the conditioning of the column blocks, and per element the
  forward error |z - z_ref| <= 64 u (M^{-1}|M||z_ref|)_i, the first-order
  bound of a solve with componentwise backward error 64 u |M| (the column
  blocks are M-matrices, so the bound is one more line solve);
* solves: at an equal number of iterations the FP64 iterates agree to 1e-10
  relative (rounding differences amplified by a handful of iterations);
  mixed precision must reach an FP64 true residual < 1e-8, computed by the
  oracle's own assembled matrix.
"""
import functools

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_1302_7193_amd as pcg  # noqa: E402
import synth_inputs as si  # noqa: E402
from _checks import column_backward_errors, line_solve_bound  # noqa: E402

U64, U32 = 2.0**-53, 2.0**-24


def make_desc(nx, ny, nz, g2=1e3, q=1.05, bcx=0, bcy=0, kh=1.0, dx=None, dy=None):
    d = pcg.pcg_desc_from_ratio(nx, ny, nz, q, g2, 0)
    d.bc_x, d.bc_y = bcx, bcy
    if dx is not None:
        d.dx = dx
    if dy is not None:
        d.dy = dy
    d.k_h = kh
    return d


def grid_of(d):
    return oracle.Grid(d.nx, d.ny, d.nz, d.dx, d.dy, d.height, d.grading, d.k_h, d.k_v,
                       d.bc_x == 1, d.bc_y == 1)


GRIDS = {
    "64x64x32-dir": lambda: make_desc(64, 64, 32, 1e4),
    "13x7x33-dir-ragged": lambda: make_desc(13, 7, 33, 1e3),
    "9x5x17-per": lambda: make_desc(9, 5, 17, 1e5, bcx=1, bcy=1),
    "6x11x100-mixedbc": lambda: make_desc(6, 11, 100, 1e2, q=1.1, bcx=1, bcy=0, dx=0.3, dy=0.2),
    "5x4x1-single-level": lambda: make_desc(5, 4, 1, 1e3),
    "1x1x40-single-column": lambda: make_desc(1, 1, 40, 1e4),
    "1x9x8-one-row": lambda: make_desc(1, 9, 8, 1e3),
    "7x6x1024-tall": lambda: make_desc(7, 6, 1024, 1e4),
    "3x3x7-per-min": lambda: make_desc(3, 3, 7, 1e3, bcx=1, bcy=1),
}
DT = {pcg.PCG_F64: (torch.float64, U64), pcg.PCG_F32: (torch.float32, U32)}


def cuda(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


@pytest.mark.parametrize("name", list(GRIDS))
@pytest.mark.parametrize("dtype", [pcg.PCG_F64, pcg.PCG_F32])
def test_apply_matches_assembled_operator(name, dtype):
    d = GRIDS[name]()
    print("apply", name, dtype, flush=True)
    p = pcg.Problem(d)
    tdt, u = DT[dtype]
    x = si.uniform_pm1(11, p.n)
    xt = cuda(x, tdt)
    y = torch.full_like(xt, float("nan"))
    pcg.pcg_apply(p, dtype, xt, y)
    torch.cuda.synchronize()
    A = oracle.assemble(grid_of(d))
    xr = xt.double().cpu().numpy()           # the input the GPU actually saw
    ref = A.matvec(xr)
    absA = oracle.CSR(A.n, A.row_ptr, A.col, np.abs(A.val))
    bound = 64 * u * absA.matvec(np.abs(xr)) + 1e-300
    err = np.abs(y.double().cpu().numpy() - ref)
    assert np.all(err <= bound), (err / bound).max()


@pytest.mark.parametrize("name", list(GRIDS))
@pytest.mark.parametrize("dtype", [pcg.PCG_F64, pcg.PCG_F32])
def test_line_preconditioner_matches_oracle(name, dtype):
    d = GRIDS[name]()
    print("precond", name, dtype, flush=True)
    p = pcg.Problem(d)
    tdt, u = DT[dtype]
    r = cuda(si.uniform_pm1(12, p.n), tdt)
    z = torch.full_like(r, float("nan"))
    pcg.pcg_precond(p, dtype, r, z)
    torch.cuda.synchronize()
    A = oracle.assemble(grid_of(d))
    M = oracle.line_blocks(A, d.nz)
    rr, zz = r.double().cpu().numpy(), z.double().cpu().numpy()
    back = column_backward_errors(M, zz, rr, d.nz).max()
    assert back <= 64 * u * (4 if dtype == pcg.PCG_F32 else 1), back
    check_line_solve(M, rr, zz, u)


def check_line_solve(M, rr, zz, u, what=""):
    """Every element of the GPU's z within the componentwise forward bound
    of the oracle's column solves of the same r."""
    zo = oracle.line_solve(M, rr)
    bound = line_solve_bound(M, zo, u, 64) + 1e-300
    ratio = (np.abs(zz - zo) / bound).max()
    print("line solve %s: max |z - z_ref| / bound = %.3f" % (what, ratio), flush=True)
    assert ratio <= 1.0, (what, ratio)


@pytest.mark.parametrize("name", ["64x64x32-dir", "13x7x33-dir-ragged", "9x5x17-per",
                                  "6x11x100-mixedbc", "5x4x1-single-level", "1x1x40-single-column"])
@pytest.mark.parametrize("dtype", [pcg.PCG_F64, pcg.PCG_F32])
def test_csr_comparator_matches_oracle(name, dtype):
    d = GRIDS[name]()
    print("csr", name, dtype, flush=True)
    p = pcg.Problem(d)
    tdt, u = DT[dtype]
    A = oracle.assemble(grid_of(d))
    nnz = A.val.size
    vs = 8 if dtype == pcg.PCG_F64 else 4
    al = lambda v: (v + 255) // 256 * 256
    assert pcg.pcg_csr_bytes(p, dtype) == al(vs * nnz) + al(4 * nnz) + al(4 * (p.n + 1))
    buf = torch.zeros(pcg.pcg_csr_bytes(p, dtype), dtype=torch.uint8, device="cuda")
    pcg.pcg_csr_build(p, dtype, buf)
    x = cuda(si.uniform_pm1(13, p.n), tdt)
    y = torch.empty_like(x)
    pcg.pcg_csr_apply(p, dtype, buf, x, y)
    torch.cuda.synchronize()
    xr = x.double().cpu().numpy()
    absA = oracle.CSR(A.n, A.row_ptr, A.col, np.abs(A.val))
    err = np.abs(y.double().cpu().numpy() - A.matvec(xr))
    assert np.all(err <= 64 * u * absA.matvec(np.abs(xr)) + 1e-300)
    rowp = buf[al(vs * nnz) + al(4 * nnz):].view(torch.int32)[: p.n + 1].cpu().numpy()
    np.testing.assert_array_equal(rowp, A.row_ptr.astype(np.int32))


SOLVE_GRIDS = ["64x64x32-dir", "13x7x33-dir-ragged", "9x5x17-per", "6x11x100-mixedbc",
               "5x4x1-single-level", "1x1x40-single-column", "3x3x7-per-min"]


def oracle_run(d, b, rtol=1e-8, max_iter=10000):
    A = oracle.assemble(grid_of(d))
    M = oracle.line_blocks(A, d.nz)
    return A, oracle.pcg(A, M, b, rtol=rtol, max_iter=max_iter)


def gpu_solve(d, b, **kw):
    p = pcg.Problem(d)
    o = pcg.pcg_default_opts(**kw)
    bt = cuda(b)
    x = torch.zeros_like(bt)
    ws = pcg.workspace(p, o)
    st, res = pcg.pcg_solve(p, bt, x, ws, o)
    torch.cuda.synchronize()
    return x.cpu().numpy(), st, res


@pytest.mark.parametrize("name", SOLVE_GRIDS)
@pytest.mark.parametrize("fused", [1, 0])
def test_fp64_solve_equal_iterations(name, fused):
    d = GRIDS[name]()
    print("solve", name, "fused" if fused else "unfused", flush=True)
    b = si.rhs_uniform(d.nx, d.ny, d.nz, 3)
    A, ref = oracle_run(d, b, rtol=1e-8)
    k = ref["iterations"]
    x, st, res = gpu_solve(d, b, rtol=0.0, max_iter=k, fused=fused, graph_chunk=3)
    assert res["iterations"] == k and st == pcg.PCG_E_NOCONV
    err = np.linalg.norm(x - ref["x"]) / np.linalg.norm(ref["x"])
    assert err <= 1e-10, err


@pytest.mark.parametrize("name", SOLVE_GRIDS)
@pytest.mark.parametrize("fused", [1, 0])
def test_fp64_solve_converges_like_oracle(name, fused):
    d = GRIDS[name]()
    print("converge", name, fused, flush=True)
    b = si.rhs_uniform(d.nx, d.ny, d.nz, 4)
    A, ref = oracle_run(d, b, rtol=1e-8)
    x, st, res = gpu_solve(d, b, rtol=1e-8, fused=fused, true_residual=1)
    assert st == pcg.PCG_OK
    assert abs(res["iterations"] - ref["iterations"]) <= 1
    true = oracle.residual_norm(A, b, x) / np.linalg.norm(b)
    assert true < 1.05e-8, true
    # both residuals carry an absolute rounding floor of ~n u ||A|| ||x|| / ||b||
    assert abs(res["rel_res_true"] - true) <= 1e-3 * true + 1e-13


@pytest.mark.parametrize("name", SOLVE_GRIDS)
@pytest.mark.parametrize("gc", [3, 0])
def test_fp64_zero_start_equal_iterations(name, gc):
    """x0 = 0 without reading x (x filled with NaN), the benchmark's path:
    kernel A's first launch leaves u unwritten and does not store p = z,
    kernel B's first launch does not copy b into r; stopped after one, two
    and all iterations (the exit correction after one iteration sets
    u = alpha p), graph chunks and direct launches, against the oracle."""
    d = GRIDS[name]()
    print("zero start", name, gc, flush=True)
    b = si.rhs_uniform(d.nx, d.ny, d.nz, 5)
    A = oracle.assemble(grid_of(d))
    M = oracle.line_blocks(A, d.nz)
    k = oracle.pcg(A, M, b, rtol=1e-8)["iterations"]
    p = pcg.Problem(d)
    bt = cuda(b)
    for kk in sorted({1, min(2, k), k}):
        ref = oracle.pcg(A, M, b, rtol=0.0, max_iter=kk)
        o = pcg.pcg_default_opts(rtol=0.0, max_iter=kk, x0_zero=1, graph_chunk=gc)
        x = torch.full_like(bt, float("nan"))
        st, res = pcg.pcg_solve(p, bt, x, pcg.workspace(p, o), o)
        assert res["iterations"] == ref["iterations"], (kk, res["iterations"])
        xs = x.cpu().numpy()
        err = np.linalg.norm(xs - ref["x"]) / max(np.linalg.norm(ref["x"]), 1e-300)
        assert err <= 1e-10, (kk, err)
        assert np.array_equal(b, bt.cpu().numpy())    # b is never written


def test_fused_and_unfused_iterates_agree():
    d = GRIDS["64x64x32-dir"]()
    b = si.rhs_uniform(64, 64, 32, 5)
    xf, _, rf = gpu_solve(d, b, rtol=0.0, max_iter=4, fused=1)
    xu, _, ru = gpu_solve(d, b, rtol=0.0, max_iter=4, fused=0)
    assert rf["iterations"] == ru["iterations"] == 4
    assert np.linalg.norm(xf - xu) <= 1e-11 * np.linalg.norm(xu)


def test_graph_and_direct_launches_bitwise_equal():
    d = GRIDS["13x7x33-dir-ragged"]()
    b = si.rhs_uniform(d.nx, d.ny, d.nz, 6)
    xg, _, rg = gpu_solve(d, b, graph_chunk=2)
    xd, _, rd = gpu_solve(d, b, graph_chunk=0)
    xp, _, rp = gpu_solve(d, b, graph_chunk=0, profile=1)
    # profiled graph chunks: event nodes inside the graph, several replays
    xq, _, rq = gpu_solve(d, b, graph_chunk=2, profile=1)
    # kernel A timed alone, graph chunks and direct launches
    xa, _, ra = gpu_solve(d, b, graph_chunk=2, profile=2)
    xe, _, re_ = gpu_solve(d, b, graph_chunk=0, profile=2)
    assert rg["iterations"] == rd["iterations"] == rp["iterations"] == rq["iterations"]
    assert ra["iterations"] == re_["iterations"] == rg["iterations"]
    for x in (xd, xp, xq, xa, xe):
        assert np.array_equal(xg, x)
    for r in (rp, rq):
        assert r["n_apply_kernel"] == r["iterations"] and r["n_precond_kernel"] == r["iterations"] + 1
        assert r["ms_apply_kernel"] > 0 and r["ms_precond_kernel"] > 0
    for r in (ra, re_):
        assert r["n_apply_kernel"] == r["iterations"] and r["n_precond_kernel"] == 0
        assert r["ms_apply_kernel"] > 0 and r["ms_precond_kernel"] == 0


def test_repeated_solves_bitwise_reproducible():
    d = GRIDS["64x64x32-dir"]()
    p = pcg.Problem(d)
    o = pcg.pcg_default_opts()
    b = cuda(si.rhs_uniform(64, 64, 32, 7))
    ws = pcg.workspace(p, o)
    outs = []
    for _ in range(6):
        x = torch.zeros_like(b)
        pcg.pcg_solve(p, b, x, ws, o)
        outs.append(x.cpu())
    for o2 in outs[1:]:
        assert torch.equal(outs[0], o2)


def test_zero_rhs_and_failure_statuses():
    d = GRIDS["13x7x33-dir-ragged"]()
    n = d.nx * d.ny * d.nz
    x, st, res = gpu_solve(d, np.zeros(n))
    assert st == pcg.PCG_OK and res["iterations"] == 0 and not x.any()
    b = si.rhs_uniform(d.nx, d.ny, d.nz, 8)
    b[17] = np.nan
    x, st, res = gpu_solve(d, b)
    assert st == pcg.PCG_E_BREAKDOWN
    x, st, res = gpu_solve(d, si.rhs_uniform(d.nx, d.ny, d.nz, 8), max_iter=1)
    assert st == pcg.PCG_E_NOCONV and res["iterations"] == 1 and res["rel_res_recursive"] < 1
    p = pcg.Problem(d)
    o = pcg.pcg_default_opts()
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        pcg.pcg_solve(p, cuda(b), torch.zeros(n, dtype=torch.float64, device="cuda"), small, o)
    bt, xt = cuda(b), torch.zeros(n, dtype=torch.float64, device="cuda")   # keep both alive
    st = pcg._lib.pcg_solve(p.handle, bt.data_ptr(), xt.data_ptr(), small.data_ptr(), 16, None,
                            pcg.ctypes.byref(pcg.pcg_result()), None)
    assert st == pcg.PCG_E_NOMEM
    st = pcg._lib.pcg_solve(p.handle, bt.data_ptr(), bt.data_ptr(), small.data_ptr(), 16, None,
                            pcg.ctypes.byref(pcg.pcg_result()), None)
    assert st == pcg.PCG_E_INVALID and "overlap" in pcg.pcg_last_error()
    st = pcg._lib.pcg_solve(p.handle, bt.data_ptr() + 8, xt.data_ptr(), small.data_ptr(), 16,
                            None, pcg.ctypes.byref(pcg.pcg_result()), None)
    assert st == pcg.PCG_E_INVALID and "aligned" in pcg.pcg_last_error()


def test_no_horizontal_coupling_converges_in_one_iteration():
    d = make_desc(9, 7, 24, 1e3, kh=0.0)
    x, st, res = gpu_solve(d, si.rhs_uniform(9, 7, 24, 9), rtol=1e-12)
    assert st == pcg.PCG_OK and res["iterations"] == 1


@pytest.mark.parametrize("name", ["64x64x32-dir", "9x5x17-per", "6x11x100-mixedbc"])
def test_mixed_precision_reaches_fp64_tolerance(name):
    d = GRIDS[name]()
    print("mixed", name, flush=True)
    b = si.rhs_smooth_noise(d.nx, d.ny, d.nz, 2)
    A, ref = oracle_run(d, b, rtol=1e-12)
    x, st, res = gpu_solve(d, b, precision=pcg.PCG_PREC_MIXED, rtol=1e-8)
    assert st == pcg.PCG_OK, res
    true = oracle.residual_norm(A, b, x) / np.linalg.norm(b)
    assert true < 1e-8, true
    assert abs(res["rel_res_true"] - true) <= 1e-4 * true + 1e-13
    err = np.linalg.norm(x - ref["x"]) / np.linalg.norm(ref["x"])
    print("mixed %s: outer %d inner %d true residual %.2e error vs FP64 oracle %.2e"
          % (name, res["outer_iterations"], res["iterations"], true, err))
    assert err < 1e-6


@pytest.mark.parametrize("precision", [pcg.PCG_PREC_FP64, pcg.PCG_PREC_MIXED])
@pytest.mark.parametrize("x0z", [0, 1])
def test_batched_equals_single_solves(precision, x0z):
    d = GRIDS["13x7x33-dir-ragged"]()
    p = pcg.Problem(d)
    n = p.n
    nrhs = 5
    B = np.stack([si.rhs_uniform(d.nx, d.ny, d.nz, 100 + s) for s in range(nrhs)])
    B[2] *= 1e-3            # different scales and one zero right-hand side
    B[4] = 0.0
    o = pcg.pcg_default_opts(precision=precision, x0_zero=x0z)
    bt = cuda(B.ravel())
    x = torch.zeros_like(bt)
    ws = pcg.workspace(p, o, nrhs)
    st, res = pcg.pcg_solve_batched(p, nrhs, bt, x, ws, o)
    torch.cuda.synchronize()
    X = x.cpu().numpy().reshape(nrhs, n)
    A = oracle.assemble(grid_of(d))
    for s in range(nrhs):
        xs, sts, rs = gpu_solve(d, B[s], precision=precision, x0_zero=x0z)
        assert res[s]["status"] == sts == pcg.PCG_OK
        assert res[s]["iterations"] == rs["iterations"]
        np.testing.assert_array_equal(X[s], xs)
        if B[s].any():
            assert oracle.residual_norm(A, B[s], X[s]) / np.linalg.norm(B[s]) < 1.05e-8


@functools.lru_cache(maxsize=1)
def _periodic_512():
    """The 512 x 512 x 128 periodic workload (anisotropy 1e5): descriptor,
    oracle grid, assembled matrix and line blocks (assembled once)."""
    d = make_desc(512, 512, 128, 1e5, bcx=1, bcy=1)
    g = grid_of(d)
    A = oracle.assemble(g)
    return d, g, A, oracle.line_blocks(A, 128)


def test_full_size_periodic_workload_sampled():
    """512 x 512 x 128 periodic, anisotropy 1e5: operator rows sampled against
    the oracle's row formula, and the converged solution's residual from the
    oracle's assembled matrix."""
    d, g, A, _ = _periodic_512()
    p = pcg.Problem(d)
    n = p.n
    x = si.uniform_pm1(21, n)
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    pcg.pcg_apply(p, pcg.PCG_F64, cuda(x), y)
    yh = y.cpu().numpy()
    rng = np.random.default_rng(0)
    for _ in range(300):
        i, j, k = rng.integers(512), rng.integers(512), rng.integers(128)
        if rng.random() < 0.3:
            i = rng.choice([0, 511])
        if rng.random() < 0.3:
            k = rng.choice([0, 127])
        ref = oracle.row_apply(g, int(i), int(j), int(k), x)
        assert abs(yh[(i * 512 + j) * 128 + k] - ref) <= 1e-12 * (abs(ref) + 1e4)
    b = si.rhs_uniform(512, 512, 128, 1)
    xs, st, res = gpu_solve(d, b, true_residual=1)
    assert st == pcg.PCG_OK
    true = oracle.residual_norm(A, b, xs) / np.linalg.norm(b)
    print("512x512x128: %d iterations, true residual %.3e (GPU %.3e)"
          % (res["iterations"], true, res["rel_res_true"]))
    assert true < 1.05e-8


@pytest.mark.parametrize("dtype", [pcg.PCG_F64, pcg.PCG_F32])
def test_full_size_csr_comparator(dtype):
    """The CSR comparator at the benchmark's size (512 x 512 x 128 periodic,
    131 072 workgroups of 256 rows): every row offset equals the oracle's
    assembly and every output element the oracle's CSR product, within the
    same bound as on the small grids."""
    d, g, A, _ = _periodic_512()
    p = pcg.Problem(d)
    tdt, u = DT[dtype]
    print("full-size csr", dtype, flush=True)
    buf = torch.empty(pcg.pcg_csr_bytes(p, dtype), dtype=torch.uint8, device="cuda")
    pcg.pcg_csr_build(p, dtype, buf)
    x = cuda(si.uniform_pm1(23, p.n), tdt)
    y = torch.empty_like(x)
    pcg.pcg_csr_apply(p, dtype, buf, x, y)
    torch.cuda.synchronize()
    xr = x.double().cpu().numpy()
    bound = 64 * u * oracle.CSR(A.n, A.row_ptr, A.col, np.abs(A.val)).matvec(np.abs(xr))
    err = np.abs(y.double().cpu().numpy() - A.matvec(xr))
    assert np.all(err <= bound + 1e-300), float(np.max(err / (bound + 1e-300)))
    vs = 8 if dtype == pcg.PCG_F64 else 4
    al = lambda v: (v + 255) // 256 * 256
    nnz = A.val.size
    rowp = buf[al(vs * nnz) + al(4 * nnz):].view(torch.int32)[: p.n + 1].cpu().numpy()
    np.testing.assert_array_equal(rowp, A.row_ptr.astype(np.int32))


def test_full_size_periodic_equal_iterations():
    """The headline workload in the benchmark's launch configuration (zero
    start, adaptive HIP-graph chunks with event nodes, the committed tuning:
    one column per wavefront, nontemporal streams): the FP64 iterate after
    the oracle's iteration count equals the oracle's to 1e-10, and so does
    the iterate stopped after one and two iterations (the first launches'
    special cases).  Right-hand side U[-1, 1) from seed 1."""
    d, g, A, M = _periodic_512()
    b = si.rhs_uniform(512, 512, 128, 1)
    k = oracle.pcg(A, M, b, rtol=1e-8)["iterations"]
    p = pcg.Problem(d)
    t = pcg.pcg_get_tuning(p, pcg.PCG_F64)
    assert t.lanes_per_column == 64 and t.lanes_per_column_prec == 64, t.as_dict()
    bt = cuda(b)
    for kk in (1, 2, k):
        ref = oracle.pcg(A, M, b, rtol=0.0, max_iter=kk)
        o = pcg.pcg_default_opts(rtol=0.0, max_iter=kk, x0_zero=1, graph_chunk=-1, profile=1)
        x = torch.full_like(bt, float("nan"))
        print("512x512x128 equal iterations: %d" % kk, flush=True)
        st, res = pcg.pcg_solve(p, bt, x, pcg.workspace(p, o), o)
        assert res["iterations"] == kk
        err = np.linalg.norm(x.cpu().numpy() - ref["x"]) / np.linalg.norm(ref["x"])
        print("512x512x128 after %d iterations: rel. difference to oracle %.2e" % (kk, err))
        assert err <= 1e-10, (kk, err)


@pytest.mark.timeout(900)   # the oracle's FP64 solve of 134M unknowns takes a minute
def test_full_size_mixed_precision_1024():
    """1024 x 1024 x 128 Dirichlet, anisotropy 1e4, smooth field + 1 % noise:
    mixed precision (FP32 inner solves, FP64 refinement) at full size; the
    returned x's residual from the oracle's assembled matrix, and its error
    against the oracle's FP64 solve to 1e-12."""
    d = make_desc(1024, 1024, 128, 1e4)
    g = grid_of(d)
    b = si.rhs_smooth_noise(1024, 1024, 128, 2)
    print("1024x1024x128 mixed", flush=True)
    xs, st, res = gpu_solve(d, b, precision=pcg.PCG_PREC_MIXED, x0_zero=1)
    assert st == pcg.PCG_OK, res
    A = oracle.assemble(g)
    true = oracle.residual_norm(A, b, xs) / np.linalg.norm(b)
    print("1024x1024x128 mixed: %d inner iterations, %d refinements, true residual %.3e"
          % (res["iterations"], res["outer_iterations"], true), flush=True)
    assert true < 1e-8
    ref = oracle.pcg(A, oracle.line_blocks(A, 128), b, rtol=1e-12)
    err = np.linalg.norm(xs - ref["x"]) / np.linalg.norm(ref["x"])
    print("1024x1024x128 mixed: error against the FP64 oracle (%d iterations to 1e-12) %.3e"
          % (ref["iterations"], err))
    assert err < 1e-6


def test_full_size_batched_64_right_hand_sides():
    """64 right-hand sides (seeds 100..163) on 256 x 256 x 64 Dirichlet,
    anisotropy 1e3, in one batched mixed-precision solve: every one converged,
    eight of them checked against the oracle's assembled matrix."""
    d = make_desc(256, 256, 64, 1e3)
    p = pcg.Problem(d)
    n, nrhs = p.n, 64
    B = np.concatenate([si.rhs_uniform(256, 256, 64, 100 + s) for s in range(nrhs)])
    o = pcg.pcg_default_opts(precision=pcg.PCG_PREC_MIXED, x0_zero=1)
    bt = cuda(B)
    x = torch.empty_like(bt)
    print("batched 64 x 256x256x64", flush=True)
    st, res = pcg.pcg_solve_batched(p, nrhs, bt, x, pcg.workspace(p, o, nrhs), o)
    assert all(r["status"] == pcg.PCG_OK for r in res)
    X = x.cpu().numpy().reshape(nrhs, n)
    A = oracle.assemble(grid_of(d))
    for s in range(0, nrhs, 8):
        bs = B[s * n:(s + 1) * n]
        true = oracle.residual_norm(A, bs, X[s]) / np.linalg.norm(bs)
        assert true < 1e-8, (s, true)


# ------------------------------------------------------------ tunings --

def _lane_counts(nz):
    return [L for L in (1, 2, 4, 8, 16, 32, 64) if 16 * L >= nz]


@pytest.mark.parametrize("name", ["64x64x32-dir", "13x7x33-dir-ragged", "6x11x100-mixedbc"])
@pytest.mark.parametrize("dtype", [pcg.PCG_F64, pcg.PCG_F32])
def test_every_lane_count_and_tiny_block_caps(name, dtype):
    """Operator and line solve for every supported L, with block caps small
    enough that each workgroup walks many tiles."""
    d = GRIDS[name]()
    print("tunings", name, dtype, flush=True)
    p = pcg.Problem(d)
    tdt, u = DT[dtype]
    A = oracle.assemble(grid_of(d))
    M = oracle.line_blocks(A, d.nz)
    absA = oracle.CSR(A.n, A.row_ptr, A.col, np.abs(A.val))
    x = cuda(si.uniform_pm1(31, p.n), tdt)
    xr = x.double().cpu().numpy()
    ref = A.matvec(xr)
    bound = 64 * u * absA.matvec(np.abs(xr)) + 1e-300
    for L in _lane_counts(d.nz):
        for cap in (1, 3, 2048):
            pcg.pcg_set_tuning(p, dtype, lanes_per_column=L, block_cap=cap, reduction=1)
            y = torch.full_like(x, float("nan"))
            pcg.pcg_apply(p, dtype, x, y)
            z = torch.full_like(x, float("nan"))
            pcg.pcg_precond(p, dtype, x, z)
            torch.cuda.synchronize()
            err = np.abs(y.double().cpu().numpy() - ref)
            assert np.all(err <= bound), (L, cap, (err / bound).max())
            check_line_solve(M, xr, z.double().cpu().numpy(), u, "L=%d cap=%d" % (L, cap))


@pytest.mark.parametrize("precision", [pcg.PCG_PREC_FP64, pcg.PCG_PREC_MIXED])
def test_reduction_modes_bitwise_identical(precision):
    d = GRIDS["13x7x33-dir-ragged"]()
    b = cuda(si.rhs_uniform(d.nx, d.ny, d.nz, 41))
    outs = []
    for mode in (0, 1, 0, 1):
        for cap in (5,):
            p = pcg.Problem(d)
            for dt in (pcg.PCG_F64, pcg.PCG_F32):
                pcg.pcg_set_tuning(p, dt, block_cap=cap, reduction=mode)
            o = pcg.pcg_default_opts(precision=precision)
            x = torch.zeros_like(b)
            st, r = pcg.pcg_solve(p, b, x, pcg.workspace(p, o), o)
            assert st == pcg.PCG_OK
            outs.append((x.cpu(), r["iterations"]))
    for xo, it in outs[1:]:
        assert it == outs[0][1] and torch.equal(xo, outs[0][0])


@pytest.mark.parametrize("L,cap,mode", [(4, 1, 0), (8, 7, 1), (16, 64, 0), (64, 2048, 1)])
def test_fp64_solve_parity_under_tunings(L, cap, mode):
    d = GRIDS["6x11x100-mixedbc"]()
    b = si.rhs_uniform(d.nx, d.ny, d.nz, 42)
    A, ref = oracle_run(d, b, rtol=1e-8)
    k = ref["iterations"]
    p = pcg.Problem(d)
    if 16 * L < d.nz:
        pytest.skip("lane count too small for n_z")
    pcg.pcg_set_tuning(p, pcg.PCG_F64, lanes_per_column=L, block_cap=cap, reduction=mode)
    o = pcg.pcg_default_opts(rtol=0.0, max_iter=k)
    bt = cuda(b)
    x = torch.zeros_like(bt)
    st, r = pcg.pcg_solve(p, bt, x, pcg.workspace(p, o), o)
    assert r["iterations"] == k
    err = np.linalg.norm(x.cpu().numpy() - ref["x"]) / np.linalg.norm(ref["x"])
    assert err <= 1e-10, err


@pytest.mark.parametrize("dtype", [pcg.PCG_F64, pcg.PCG_F32])
def test_separate_launch_shapes_for_the_line_solve_kernels(dtype):
    """Kernel B (and the preconditioner alone) with its own lanes per column
    and block cap: FP64 parity with the oracle at equal iterations, mixed
    precision to the FP64 tolerance, graph and direct launches bitwise
    equal, and the preconditioner still the exact line solve."""
    d = GRIDS["6x11x100-mixedbc"]()
    b = si.rhs_uniform(d.nx, d.ny, d.nz, 45)
    A, ref = oracle_run(d, b, rtol=1e-8)
    k = ref["iterations"]
    outs = []
    for gc in (0, 3):
        p = pcg.Problem(d)
        pcg.pcg_set_tuning(p, dtype, lanes_per_column=8, block_cap=5, reduction=1,
                           lanes_per_column_prec=64, block_cap_prec=2)
        t = pcg.pcg_get_tuning(p, dtype)
        assert (t.lanes_per_column, t.block_cap, t.lanes_per_column_prec, t.block_cap_prec) == \
            (8, 5, 64, 2)
        if dtype == pcg.PCG_F64:
            o = pcg.pcg_default_opts(rtol=0.0, max_iter=k, graph_chunk=gc)
        else:
            o = pcg.pcg_default_opts(precision=pcg.PCG_PREC_MIXED, graph_chunk=gc)
        bt = cuda(b)
        x = torch.zeros_like(bt)
        st, r = pcg.pcg_solve(p, bt, x, pcg.workspace(p, o), o)
        outs.append(x.cpu())
        if dtype == pcg.PCG_F64:
            assert r["iterations"] == k
            err = np.linalg.norm(x.cpu().numpy() - ref["x"]) / np.linalg.norm(ref["x"])
            assert err <= 1e-10, err
        else:
            assert st == pcg.PCG_OK
            assert oracle.residual_norm(A, b, x.cpu().numpy()) / np.linalg.norm(b) < 1e-8
    assert torch.equal(outs[0], outs[1])
    tdt, u = DT[dtype]
    r = cuda(si.uniform_pm1(46, p.n), tdt)
    z = torch.full_like(r, float("nan"))
    pcg.pcg_precond(p, dtype, r, z)
    torch.cuda.synchronize()
    M = oracle.line_blocks(A, d.nz)
    check_line_solve(M, r.double().cpu().numpy(), z.double().cpu().numpy(), u, "L_b=64")


def test_set_tuning_rejects_bad_values():
    p = pcg.Problem(GRIDS["7x6x1024-tall"]())
    for bad in (dict(lanes_per_column=32), dict(lanes_per_column=3), dict(block_cap=0),
                dict(block_cap=70000), dict(reduction=2), dict(lanes_per_column_prec=16),
                dict(block_cap_prec=0)):
        with pytest.raises(pcg.PCGError):
            pcg.pcg_set_tuning(p, pcg.PCG_F64, **bad)
    t = pcg.pcg_get_tuning(p, pcg.PCG_F64)
    assert t.lanes_per_column == 64


@pytest.mark.parametrize("dtype,nrhs", [(pcg.PCG_F64, 1), (pcg.PCG_F32, 3)])
def test_autotune_picks_a_valid_tuning_and_solves(dtype, nrhs):
    d = GRIDS["64x64x32-dir"]()
    p = pcg.Problem(d)
    t = pcg.pcg_autotune(p, dtype, nrhs)
    assert 16 * t.lanes_per_column >= d.nz and t.block_cap >= 1 and t.reduction in (0, 1)
    assert pcg.pcg_get_tuning(p, dtype).as_dict() == t.as_dict()
    b = si.rhs_uniform(d.nx, d.ny, d.nz, 43)
    prec = pcg.PCG_PREC_FP64 if dtype == pcg.PCG_F64 else pcg.PCG_PREC_MIXED
    o = pcg.pcg_default_opts(precision=prec)
    bt = cuda(b)
    x = torch.zeros_like(bt)
    st, r = pcg.pcg_solve(p, bt, x, pcg.workspace(p, o), o)
    assert st == pcg.PCG_OK
    A = oracle.assemble(grid_of(d))
    assert oracle.residual_norm(A, b, x.cpu().numpy()) / np.linalg.norm(b) < 1.05e-8


def test_mixed_precision_zero_start_ignores_x():
    d = GRIDS["9x5x17-per"]()
    b = si.rhs_smooth_noise(d.nx, d.ny, d.nz, 2)
    p = pcg.Problem(d)
    o = pcg.pcg_default_opts(precision=pcg.PCG_PREC_MIXED, x0_zero=1)
    bt = cuda(b)
    x = torch.full_like(bt, 1e30)          # garbage that must not be read
    st, r = pcg.pcg_solve(p, bt, x, pcg.workspace(p, o), o)
    assert st == pcg.PCG_OK
    A = oracle.assemble(grid_of(d))
    true = oracle.residual_norm(A, b, x.cpu().numpy()) / np.linalg.norm(b)
    assert true < 1e-8 and abs(r["r0_norm"] - np.linalg.norm(b)) < 1e-12 * np.linalg.norm(b)
    o.precision = pcg.PCG_PREC_FP64
    x.fill_(1e30)
    st, r = pcg.pcg_solve(p, bt, x, pcg.workspace(p, o), o)
    assert st == pcg.PCG_OK
    assert oracle.residual_norm(A, b, x.cpu().numpy()) / np.linalg.norm(b) < 1.05e-8


def test_tuning_cache_entry_applies_unless_set_explicitly(tmp_path):
    """A cache entry for a shape changes the launch parameters of new problems
    of that shape (solve bitwise equal to the same tuning set explicitly);
    an explicit setting wins over the cache."""
    d = make_desc(23, 19, 61, 1e4)
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    f = tmp_path / "cache.txt"
    f.write_text(f"{arch} uniform 23 19 61 0 1 8 3 0\n")
    pcg.pcg_tuning_cache_load(str(f))
    b = cuda(si.rhs_uniform(d.nx, d.ny, d.nz, 44))
    o = pcg.pcg_default_opts()

    def run(p):
        x = torch.zeros_like(b)
        st, r = pcg.pcg_solve(p, b, x, pcg.workspace(p, o), o)
        assert st == pcg.PCG_OK
        return x.cpu(), r["iterations"]

    cached = pcg.Problem(d)
    t = pcg.pcg_get_tuning(cached, pcg.PCG_F64)
    assert (t.lanes_per_column, t.block_cap, t.reduction) == (8, 3, 0)
    explicit = pcg.Problem(d)
    pcg.pcg_set_tuning(explicit, pcg.PCG_F64, lanes_per_column=8, block_cap=3, reduction=0)
    xc, ic = run(cached)
    xe, ie = run(explicit)
    assert ic == ie and torch.equal(xc, xe)
    pcg.pcg_set_tuning(cached, pcg.PCG_F64, lanes_per_column=64, block_cap=16384, reduction=1)
    t = pcg.pcg_get_tuning(cached, pcg.PCG_F64)
    assert (t.lanes_per_column, t.block_cap, t.reduction) == (64, 16384, 1)


# ------------------------------------------- argument changes and edges --

@pytest.mark.parametrize("precision", [pcg.PCG_PREC_FP64, pcg.PCG_PREC_MIXED])
def test_new_rhs_with_same_x_and_workspace_replays_no_stale_graph(precision):
    """Two solves on one problem, x and workspace with different right-hand
    sides (zero start, graph chunks of the same length): the second must use
    its own b, which kernel B reads inside the graph."""
    d = GRIDS["13x7x33-dir-ragged"]()
    p = pcg.Problem(d)
    A = oracle.assemble(grid_of(d))
    M = oracle.line_blocks(A, d.nz)
    b1 = si.rhs_uniform(d.nx, d.ny, d.nz, 51)
    b2 = si.rhs_uniform(d.nx, d.ny, d.nz, 52)
    k = oracle.pcg(A, M, b2, rtol=1e-8)["iterations"]
    if precision == pcg.PCG_PREC_FP64:
        o = pcg.pcg_default_opts(rtol=0.0, max_iter=k, x0_zero=1, graph_chunk=3)
    else:
        o = pcg.pcg_default_opts(precision=precision, x0_zero=1, graph_chunk=3)
    ws = pcg.workspace(p, o)
    x = torch.empty(p.n, dtype=torch.float64, device="cuda")
    outs = []
    for b in (b1, b2):
        bt = cuda(b)                       # a new buffer for each right-hand side
        x.fill_(float("nan"))
        st, res = pcg.pcg_solve(p, bt, x, ws, o)
        outs.append((x.cpu().numpy(), res))
        del bt
    x2, res2 = outs[1]
    if precision == pcg.PCG_PREC_FP64:
        ref = oracle.pcg(A, M, b2, rtol=0.0, max_iter=k)
        err = np.linalg.norm(x2 - ref["x"]) / np.linalg.norm(ref["x"])
        assert res2["iterations"] == k and err <= 1e-10, err
    else:
        assert res2["status"] == pcg.PCG_OK
        assert oracle.residual_norm(A, b2, x2) / np.linalg.norm(b2) < 1e-8
    # the same again on fresh problem: bitwise the same result
    p2 = pcg.Problem(d)
    bt = cuda(b2)
    xf = torch.full_like(bt, float("nan"))
    pcg.pcg_solve(p2, bt, xf, pcg.workspace(p2, o), o)
    assert np.array_equal(xf.cpu().numpy(), x2)


def test_many_solution_buffers_evict_graphs_and_stay_exact():
    """More distinct solution buffers than the graph cache holds: every
    solve (new graphs, evicted graphs, re-instantiated ones) gives the
    bitwise same result."""
    d = GRIDS["13x7x33-dir-ragged"]()
    p = pcg.Problem(d)
    o = pcg.pcg_default_opts(x0_zero=1, graph_chunk=2)
    bt = cuda(si.rhs_uniform(d.nx, d.ny, d.nz, 53))
    ws = pcg.workspace(p, o)
    xs = [torch.empty_like(bt) for _ in range(24)]
    first = None
    for rep in range(2):
        for x in xs:
            x.fill_(float("nan"))
            st, r = pcg.pcg_solve(p, bt, x, ws, o)
            assert st == pcg.PCG_OK
            if first is None:
                first = x.cpu()
            assert torch.equal(x.cpu(), first)


@pytest.mark.parametrize("nrhs", [1, 3])
def test_mixed_precision_zero_rhs_writes_zero(nrhs):
    """Mixed precision from a zero start: a right-hand side that meets the
    exit test at its first residual (here b = 0) still gets x = 0 written,
    alone and in a batch whose other right-hand sides iterate."""
    d = GRIDS["13x7x33-dir-ragged"]()
    p = pcg.Problem(d)
    n = p.n
    B = np.stack([si.rhs_uniform(d.nx, d.ny, d.nz, 60 + s) for s in range(nrhs)])
    B[nrhs // 2] = 0.0
    o = pcg.pcg_default_opts(precision=pcg.PCG_PREC_MIXED, x0_zero=1)
    bt = cuda(B.ravel())
    x = torch.full_like(bt, float("nan"))
    st, res = pcg.pcg_solve_batched(p, nrhs, bt, x, pcg.workspace(p, o, nrhs), o)
    X = x.cpu().numpy().reshape(nrhs, n)
    A = oracle.assemble(grid_of(d))
    for s in range(nrhs):
        assert res[s]["status"] == pcg.PCG_OK, (s, res[s])
        if B[s].any():
            assert oracle.residual_norm(A, B[s], X[s]) / np.linalg.norm(B[s]) < 1e-8
        else:
            assert res[s]["iterations"] == 0 and np.array_equal(X[s], np.zeros(n)), s
    # atol above ||b||: done at the first residual, x = 0
    o = pcg.pcg_default_opts(precision=pcg.PCG_PREC_MIXED, x0_zero=1,
                             atol=2 * np.linalg.norm(B[0]) + 1.0)
    x = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    st, r = pcg.pcg_solve(p, cuda(B[0]), x, pcg.workspace(p, o), o)
    assert st == pcg.PCG_OK and r["iterations"] == 0 and not x.cpu().numpy().any()


def test_partially_overlapping_buffers_are_rejected():
    """Outputs that share bytes with an input (other than the in-place line
    solve) are rejected before any launch."""
    d = GRIDS["13x7x33-dir-ragged"]()
    p = pcg.Problem(d)
    n = p.n
    buf = torch.zeros(2 * n + 64, dtype=torch.float64, device="cuda")
    x, y = buf[:n], buf[16:16 + n]          # y starts 128 bytes into x
    lib, F64 = pcg._lib, pcg.PCG_F64
    assert lib.pcg_apply(p.handle, F64, x.data_ptr(), y.data_ptr(), None) == pcg.PCG_E_INVALID
    assert "overlap" in pcg.pcg_last_error()
    assert lib.pcg_precond(p.handle, F64, x.data_ptr(), y.data_ptr(), None) == pcg.PCG_E_INVALID
    assert lib.pcg_rbgs_precond(p.handle, F64, x.data_ptr(), y.data_ptr(), None) == pcg.PCG_E_INVALID
    # the line solve in place is allowed and equals the out-of-place one
    r = cuda(si.uniform_pm1(70, n))
    z = torch.empty_like(r)
    pcg.pcg_precond(p, F64, r, z)
    assert lib.pcg_precond(p.handle, F64, r.data_ptr(), r.data_ptr(), None) == pcg.PCG_OK
    torch.cuda.synchronize()
    assert torch.equal(r, z)
    csr = torch.zeros(pcg.pcg_csr_bytes(p, F64), dtype=torch.uint8, device="cuda")
    pcg.pcg_csr_build(p, F64, csr)
    assert lib.pcg_csr_apply(p.handle, F64, csr.data_ptr(), x.data_ptr(), y.data_ptr(),
                             None) == pcg.PCG_E_INVALID
    assert lib.pcg_csr_apply(p.handle, F64, csr.data_ptr(), x.data_ptr(), csr.data_ptr() + 256,
                             None) == pcg.PCG_E_INVALID
    o = pcg.pcg_default_opts()
    ws = pcg.workspace(p, o)
    res = pcg.pcg_result()
    st = lib.pcg_solve(p.handle, x.data_ptr(), y.data_ptr(), ws.data_ptr(), ws.numel(), None,
                       pcg.ctypes.byref(res), None)
    assert st == pcg.PCG_E_INVALID and "overlap" in pcg.pcg_last_error()
    # a workspace that starts inside x (all of it inside one allocation, so
    # nothing would be out of bounds even unchecked)
    big = torch.zeros(ws.numel() // 8 + 2 * n + 64, dtype=torch.float64, device="cuda")
    b2, x2 = big[:n], big[n + 32:2 * n + 32]
    st = lib.pcg_solve(p.handle, b2.data_ptr(), x2.data_ptr(), x2.data_ptr() + 8 * 64,
                       ws.numel(), None, pcg.ctypes.byref(res), None)
    assert st == pcg.PCG_E_INVALID and "workspace" in pcg.pcg_last_error()
