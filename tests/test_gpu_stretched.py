"""Stretched horizontal grids on the GPU, through the C ABI, against the
oracle's assembly with per-index cell widths.

The kernels rebuild |T| and alpha_{T,T'} per column from the widths and
factorise every column block in the kernel (a scan of 2x2 pivot maps across
the lanes of a column), so these tests cover: the operator and the
preconditioner for every lane count and several grids (ragged n_z,
periodic and Dirichlet sides, strong width contrasts), the CSR comparator,
FP64 solves at equal iteration counts, mixed precision to the FP64
tolerance, batched solves, and constant widths against the uniform path.
Tolerances as in test_gpu_parity.py."""
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
DT = {pcg.PCG_F64: (torch.float64, U64), pcg.PCG_F32: (torch.float32, U32)}


def case(nx, ny, nz, g2, bcx, bcy, xw, yw, q=1.05, kh=1.0):
    d = pcg.pcg_desc_from_ratio(nx, ny, nz, q, g2, 0)
    d.bc_x, d.bc_y, d.k_h = bcx, bcy, kh
    return d, np.asarray(xw, dtype=np.float64), np.asarray(yw, dtype=np.float64)


CASES = {
    "40x36x64-sine-dir": lambda: case(40, 36, 64, 1e4, 0, 0, si.widths_sine(40), si.widths_sine(36, 0.3)),
    "13x7x33-random-ragged": lambda: case(13, 7, 33, 1e3, 0, 0, si.widths_random(13, 1, 0.2, 3.0),
                                          si.widths_random(7, 2)),
    "9x5x17-per-random": lambda: case(9, 5, 17, 1e5, 1, 1, si.widths_random(9, 3), si.widths_sine(5, 0.6)),
    "6x11x100-mixedbc-graded": lambda: case(6, 11, 100, 1e2, 1, 0, si.widths_sine(6),
                                            si.widths_graded(11, 1.5, 0.7), q=1.1),
    "16x16x128-graded-weak": lambda: case(16, 16, 128, 1e1, 0, 0, si.widths_graded(16, 1.3),
                                          si.widths_graded(16, 1.3)),
    "5x4x1-single-level": lambda: case(5, 4, 1, 1e3, 0, 0, si.widths_random(5, 4), si.widths_random(4, 5)),
    "7x6x1024-tall": lambda: case(7, 6, 1024, 1e4, 0, 1, si.widths_random(7, 6), si.widths_sine(6)),
}


def grid_of(d, xw, yw):
    return oracle.Grid(d.nx, d.ny, d.nz, d.dx, d.dy, d.height, d.grading, d.k_h, d.k_v,
                       d.bc_x == 1, d.bc_y == 1, tuple(xw), tuple(yw))


def cuda(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def check_apply(p, d, xw, yw, dtype, seed=11):
    tdt, u = DT[dtype]
    xt = cuda(si.uniform_pm1(seed, p.n), tdt)
    y = torch.full_like(xt, float("nan"))
    pcg.pcg_apply(p, dtype, xt, y)
    torch.cuda.synchronize()
    A = oracle.assemble(grid_of(d, xw, yw))
    xr = xt.double().cpu().numpy()
    absA = oracle.CSR(A.n, A.row_ptr, A.col, np.abs(A.val))
    bound = 64 * u * absA.matvec(np.abs(xr)) + 1e-300
    err = np.abs(y.double().cpu().numpy() - A.matvec(xr))
    assert np.all(err <= bound), (err / bound).max()


def check_precond(p, d, xw, yw, dtype, seed=12):
    tdt, u = DT[dtype]
    r = cuda(si.uniform_pm1(seed, p.n), tdt)
    z = torch.full_like(r, float("nan"))
    pcg.pcg_precond(p, dtype, r, z)
    torch.cuda.synchronize()
    M = oracle.line_blocks(oracle.assemble(grid_of(d, xw, yw)), d.nz)
    rr, zz = r.double().cpu().numpy(), z.double().cpu().numpy()
    back = column_backward_errors(M, zz, rr, d.nz).max()
    assert back <= 64 * u * (4 if dtype == pcg.PCG_F32 else 1), back
    # every element within the componentwise forward bound of the column
    # solves; c = 256 rather than the 64 of the class-factor path: here the
    # kernel also factorises every column, its pivots coming from a scan of
    # rounded 2 x 2 products over up to 1024 levels, which adds their
    # rounding to the backward error of the substitutions
    zo = oracle.line_solve(M, rr)
    ratio = (np.abs(zz - zo) / (line_solve_bound(M, zo, u, 256) + 1e-300)).max()
    print("stretched line solve: max |z - z_ref| / bound = %.3f" % ratio)
    assert ratio <= 1.0, ratio


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("dtype", [pcg.PCG_F64, pcg.PCG_F32])
def test_apply_matches_oracle(name, dtype):
    d, xw, yw = CASES[name]()
    print("stretched apply", name, dtype, flush=True)
    check_apply(pcg.Problem(d, xw, yw), d, xw, yw, dtype)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("dtype", [pcg.PCG_F64, pcg.PCG_F32])
def test_preconditioner_matches_oracle(name, dtype):
    d, xw, yw = CASES[name]()
    print("stretched precond", name, dtype, flush=True)
    check_precond(pcg.Problem(d, xw, yw), d, xw, yw, dtype)


@pytest.mark.parametrize("name", ["13x7x33-random-ragged", "16x16x128-graded-weak", "7x6x1024-tall"])
@pytest.mark.parametrize("dtype", [pcg.PCG_F64, pcg.PCG_F32])
def test_every_lane_count(name, dtype):
    d, xw, yw = CASES[name]()
    print("stretched lanes", name, dtype, flush=True)
    L = 1
    while L <= 64:
        if 16 * L >= d.nz:
            for cap in (1, 7, 4096):
                p = pcg.Problem(d, xw, yw)
                pcg.pcg_set_tuning(p, dtype, lanes_per_column=L, block_cap=cap, reduction=1)
                check_precond(p, d, xw, yw, dtype, seed=L + cap)
                check_apply(p, d, xw, yw, dtype, seed=L + cap)
        L *= 2


@pytest.mark.parametrize("dtype", [pcg.PCG_F64, pcg.PCG_F32])
def test_csr_comparator_matches_oracle(dtype):
    d, xw, yw = CASES["9x5x17-per-random"]()
    p = pcg.Problem(d, xw, yw)
    tdt, u = DT[dtype]
    A = oracle.assemble(grid_of(d, xw, yw))
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


def solve(d, xw, yw, b, **kw):
    p = pcg.Problem(d, xw, yw)
    o = pcg.pcg_default_opts(**kw)
    bt = cuda(b)
    x = torch.zeros_like(bt)
    st, res = pcg.pcg_solve(p, bt, x, pcg.workspace(p, o), o)
    torch.cuda.synchronize()
    return x.cpu().numpy(), st, res


@pytest.mark.parametrize("name", ["40x36x64-sine-dir", "13x7x33-random-ragged", "9x5x17-per-random",
                                  "6x11x100-mixedbc-graded", "16x16x128-graded-weak"])
@pytest.mark.parametrize("fused", [1, 0])
def test_fp64_solve_equal_iterations(name, fused):
    d, xw, yw = CASES[name]()
    print("stretched solve", name, fused, flush=True)
    b = si.rhs_uniform(d.nx, d.ny, d.nz, 3)
    A = oracle.assemble(grid_of(d, xw, yw))
    ref = oracle.pcg(A, oracle.line_blocks(A, d.nz), b, rtol=1e-8)
    k = ref["iterations"]
    x, st, res = solve(d, xw, yw, b, rtol=0.0, max_iter=k, fused=fused, graph_chunk=3)
    assert res["iterations"] == k
    err = np.linalg.norm(x - ref["x"]) / np.linalg.norm(ref["x"])
    assert err <= 1e-10, err
    x, st, res = solve(d, xw, yw, b, rtol=1e-8, fused=fused)
    assert st == pcg.PCG_OK and abs(res["iterations"] - k) <= 1
    assert oracle.residual_norm(A, b, x) / np.linalg.norm(b) < 1.05e-8


@pytest.mark.parametrize("name", ["40x36x64-sine-dir", "6x11x100-mixedbc-graded", "16x16x128-graded-weak"])
def test_mixed_precision_reaches_fp64_tolerance(name):
    d, xw, yw = CASES[name]()
    print("stretched mixed", name, flush=True)
    b = si.rhs_smooth_noise(d.nx, d.ny, d.nz, 2)
    x, st, res = solve(d, xw, yw, b, precision=pcg.PCG_PREC_MIXED, rtol=1e-8)
    assert st == pcg.PCG_OK, res
    A = oracle.assemble(grid_of(d, xw, yw))
    true = oracle.residual_norm(A, b, x) / np.linalg.norm(b)
    assert true < 1e-8, true
    assert abs(res["rel_res_true"] - true) <= 1e-4 * true + 1e-13


def test_batched_equals_single_solves():
    d, xw, yw = CASES["13x7x33-random-ragged"]()
    p = pcg.Problem(d, xw, yw)
    nrhs = 3
    B = np.stack([si.rhs_uniform(d.nx, d.ny, d.nz, 100 + s) for s in range(nrhs)])
    o = pcg.pcg_default_opts(precision=pcg.PCG_PREC_MIXED)
    bt = cuda(B.ravel())
    x = torch.zeros_like(bt)
    st, res = pcg.pcg_solve_batched(p, nrhs, bt, x, pcg.workspace(p, o, nrhs), o)
    torch.cuda.synchronize()
    X = x.cpu().numpy().reshape(nrhs, p.n)
    for s in range(nrhs):
        xs, sts, rs = solve(d, xw, yw, B[s], precision=pcg.PCG_PREC_MIXED)
        assert res[s]["iterations"] == rs["iterations"]
        np.testing.assert_array_equal(X[s], xs)


def test_constant_widths_agree_with_uniform_grid():
    d = pcg.pcg_desc_from_ratio(24, 20, 48, 1.05, 1e3, 0)
    xw, yw = np.full(24, d.dx), np.full(20, d.dy)
    b = si.rhs_uniform(24, 20, 48, 7)
    xs, st, rs = solve(d, xw, yw, b, rtol=0.0, max_iter=6)
    p = pcg.Problem(d)
    o = pcg.pcg_default_opts(rtol=0.0, max_iter=6)
    bt = cuda(b)
    xu = torch.zeros_like(bt)
    pcg.pcg_solve(p, bt, xu, pcg.workspace(p, o), o)
    xu = xu.cpu().numpy()
    assert np.linalg.norm(xs - xu) <= 1e-12 * np.linalg.norm(xu)


def test_full_size_stretched_workload_sampled():
    """512 x 512 x 128 Dirichlet, sine-stretched in x and y (width ratio 3),
    anisotropy 1e4: operator rows sampled against the oracle's row formula
    and the converged solution's residual from the oracle's assembled
    matrix."""
    d, xw, yw = case(512, 512, 128, 1e4, 0, 0, si.widths_sine(512), si.widths_sine(512, 0.25))
    g = grid_of(d, xw, yw)
    p = pcg.Problem(d, xw, yw)
    x = si.uniform_pm1(21, p.n)
    y = torch.empty(p.n, dtype=torch.float64, device="cuda")
    pcg.pcg_apply(p, pcg.PCG_F64, cuda(x), y)
    yh = y.cpu().numpy()
    rng = np.random.default_rng(0)
    for _ in range(200):
        i, j, k = rng.integers(512), rng.integers(512), rng.integers(128)
        if rng.random() < 0.3:
            i = rng.choice([0, 511])
        ref = oracle.row_apply(g, int(i), int(j), int(k), x)
        assert abs(yh[(i * 512 + j) * 128 + k] - ref) <= 1e-12 * (abs(ref) + 1e4)
    b = si.rhs_uniform(512, 512, 128, 1)
    xs, st, res = solve(d, xw, yw, b, true_residual=1)
    assert st == pcg.PCG_OK
    A = oracle.assemble(g)
    true = oracle.residual_norm(A, b, xs) / np.linalg.norm(b)
    print("stretched 512x512x128: %d iterations, true residual %.3e" % (res["iterations"], true))
    assert true < 1.05e-8
