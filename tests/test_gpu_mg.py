"""Multigrid preconditioner on the GPU, through the C ABI, against the
oracle's V-cycle and multigrid-preconditioned CG (oracle/mg.py).

* one V-cycle (pcg_mg_precond) equals the oracle's for every level count,
  uniform and stretched grids, ragged n_z, both precisions;
* FP64 MG-PCG iterates equal the oracle's at equal iteration counts (graph
  and direct launches), converged solves meet the tolerance with the
  oracle's matrix, mixed precision reaches the FP64 tolerance;
* batched, graph, direct and profiled launches bitwise equal; served
  requests with MG equal direct solves.
Tolerances, for every column separately (the error of each column relative
to its own norm, or to the root-mean-square column norm where that is
larger): the V-cycle is a fixed linear map, computed in a different order,
so FP64 results agree to a few hundred ulps of its condition; FP32 (mixed
precision's inner solves) to 1e-4."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
import oracle.mg as omg  # noqa: E402
import paper_1302_7193_amd as pcg  # noqa: E402
import synth_inputs as si  # noqa: E402
from _checks import column_rel_errors  # noqa: E402

MG = pcg.PCG_PRECOND_MG


def desc(nx, ny, nz, g2, bcx=0, bcy=0, q=1.05):
    d = pcg.pcg_desc_from_ratio(nx, ny, nz, q, g2, 0)
    d.bc_x, d.bc_y = bcx, bcy
    return d


CASES = {
    "32x32x32-dir-1e2": lambda: (desc(32, 32, 32, 1e2), None, None),
    "64x32x33-dir-ragged-1e1": lambda: (desc(64, 32, 33, 1e1), None, None),
    "16x24x17-per-1e3": lambda: (desc(16, 24, 17, 1e3, 1, 1), None, None),
    "40x12x64-mixedbc-1e2": lambda: (desc(40, 12, 64, 1e2, 1, 0, q=1.1), None, None),
    "20x16x8-oddcoarse": lambda: (desc(20, 16, 8, 1e1), None, None),
    "32x16x128-stretched": lambda: (desc(32, 16, 128, 1e2), si.widths_sine(32),
                                    si.widths_random(16, 3)),
    "13x9x16-one-level": lambda: (desc(13, 9, 16, 1e2), None, None),
}


def grid_of(d, xw, yw):
    return oracle.Grid(d.nx, d.ny, d.nz, d.dx, d.dy, d.height, d.grading, d.k_h, d.k_v,
                       d.bc_x == 1, d.bc_y == 1, None if xw is None else tuple(xw),
                       None if yw is None else tuple(yw))


def problem(d, xw, yw):
    return pcg.Problem(d, xw, yw) if xw is not None else pcg.Problem(d)


def cuda(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("dtype", [pcg.PCG_F64, pcg.PCG_F32])
def test_vcycle_matches_oracle(name, dtype):
    d, xw, yw = CASES[name]()
    print("vcycle", name, dtype, flush=True)
    p = problem(d, xw, yw)
    g = grid_of(d, xw, yw)
    assert pcg.pcg_mg_levels(p) == len(omg.levels(g))
    tdt = torch.float64 if dtype == pcg.PCG_F64 else torch.float32
    for ml in range(1, pcg.pcg_mg_levels(p) + 1):
        r = cuda(si.uniform_pm1(50 + ml, p.n), tdt)
        z = torch.full_like(r, float("nan"))
        ws = torch.empty(pcg.pcg_mg_bytes(p, dtype, ml), dtype=torch.uint8, device="cuda")
        pcg.pcg_mg_precond(p, dtype, r, z, ws, ml)
        torch.cuda.synchronize()
        want = omg.Hierarchy(g, ml).vcycle(r.double().cpu().numpy())
        err = column_rel_errors(z.double().cpu().numpy(), want, d.nz).max()
        print("vcycle %s dtype %d levels %d: worst column error %.2e" % (name, dtype, ml, err))
        assert err <= (1e-11 if dtype == pcg.PCG_F64 else 1e-4), (ml, err)


def gpu_solve(p, b, **kw):
    o = pcg.pcg_default_opts(preconditioner=MG, **kw)
    bt = cuda(b)
    x = torch.zeros_like(bt)
    st, res = pcg.pcg_solve(p, bt, x, pcg.workspace(p, o), o)
    torch.cuda.synchronize()
    return x.cpu().numpy(), st, res


@pytest.mark.parametrize("name", ["32x32x32-dir-1e2", "64x32x33-dir-ragged-1e1",
                                  "16x24x17-per-1e3", "40x12x64-mixedbc-1e2",
                                  "32x16x128-stretched", "13x9x16-one-level"])
@pytest.mark.parametrize("gc", [3, 0])
def test_fp64_mg_pcg_equal_iterations(name, gc):
    d, xw, yw = CASES[name]()
    print("mg solve", name, gc, flush=True)
    g = grid_of(d, xw, yw)
    b = si.rhs_uniform(d.nx, d.ny, d.nz, 3)
    ref = omg.solve(g, b, rtol=1e-8)
    k = ref["iterations"]
    p = problem(d, xw, yw)
    x, st, res = gpu_solve(p, b, rtol=0.0, max_iter=k, graph_chunk=gc)
    assert res["iterations"] == k
    err = np.linalg.norm(x - ref["x"]) / np.linalg.norm(ref["x"])
    assert err <= 1e-10, err
    x, st, res = gpu_solve(p, b, rtol=1e-8, graph_chunk=gc, true_residual=1)
    assert st == pcg.PCG_OK and abs(res["iterations"] - k) <= 1
    true = oracle.residual_norm(ref["A"], b, x) / np.linalg.norm(b)
    assert true < 1.05e-8, true
    assert abs(res["rel_res_true"] - true) <= 1e-3 * true + 1e-13


@pytest.mark.parametrize("name", ["64x32x33-dir-ragged-1e1", "32x16x128-stretched"])
def test_mixed_precision_mg_reaches_fp64_tolerance(name):
    d, xw, yw = CASES[name]()
    g = grid_of(d, xw, yw)
    b = si.rhs_smooth_noise(d.nx, d.ny, d.nz, 2)
    p = problem(d, xw, yw)
    x, st, res = gpu_solve(p, b, precision=pcg.PCG_PREC_MIXED)
    assert st == pcg.PCG_OK, res
    A = oracle.assemble(g)
    assert oracle.residual_norm(A, b, x) / np.linalg.norm(b) < 1e-8


def test_mg_needs_fewer_iterations_than_line_relaxation():
    d, _, _ = CASES["64x32x33-dir-ragged-1e1"]()
    p = pcg.Problem(d)
    b = cuda(si.rhs_uniform(d.nx, d.ny, d.nz, 4))
    its = {}
    for prec in (pcg.PCG_PRECOND_LINE, MG):
        o = pcg.pcg_default_opts(preconditioner=prec)
        x = torch.zeros_like(b)
        st, r = pcg.pcg_solve(p, b, x, pcg.workspace(p, o), o)
        assert st == pcg.PCG_OK
        its[prec] = r["iterations"]
    assert its[MG] * 3 < its[pcg.PCG_PRECOND_LINE], its


def test_batched_graph_direct_profiled_bitwise_equal():
    d, _, _ = CASES["40x12x64-mixedbc-1e2"]()
    p = pcg.Problem(d)
    nrhs = 3
    B = np.stack([si.rhs_uniform(d.nx, d.ny, d.nz, 200 + s) for s in range(nrhs)])
    o = pcg.pcg_default_opts(preconditioner=MG)
    bt = cuda(B.ravel())
    x = torch.zeros_like(bt)
    st, res = pcg.pcg_solve_batched(p, nrhs, bt, x, pcg.workspace(p, o, nrhs), o)
    X = x.cpu().numpy().reshape(nrhs, p.n)
    for s in range(nrhs):
        outs = []
        for kw in (dict(graph_chunk=-1), dict(graph_chunk=0), dict(profile=1)):
            xs, sts, rs = gpu_solve(p, B[s], **kw)
            assert sts == pcg.PCG_OK and rs["iterations"] == res[s]["iterations"]
            outs.append(xs)
        for xs in outs:
            np.testing.assert_array_equal(xs, X[s])


def test_workspace_and_argument_errors():
    d, _, _ = CASES["32x32x32-dir-1e2"]()
    p = pcg.Problem(d)
    o = pcg.pcg_default_opts(preconditioner=MG)
    line = pcg.pcg_default_opts()
    assert pcg.pcg_workspace_bytes(p, o) > pcg.pcg_workspace_bytes(p, line)
    b = cuda(si.rhs_uniform(32, 32, 32, 1))
    x = torch.zeros_like(b)
    small = torch.empty(pcg.pcg_workspace_bytes(p, line), dtype=torch.uint8, device="cuda")
    with pytest.raises((pcg.PCGError, ValueError)):
        pcg.pcg_solve(p, b, x, small, o)
    with pytest.raises(pcg.PCGError):
        o2 = pcg.pcg_default_opts(preconditioner=MG, fused=0)
        pcg.pcg_solve(p, b, x, pcg.workspace(p, o), o2)
    with pytest.raises(pcg.PCGError):
        o3 = pcg.pcg_default_opts(preconditioner=7)
        pcg.pcg_solve(p, b, x, pcg.workspace(p, line), o3)


def test_served_mg_request_equals_direct_solve():
    d = desc(64, 64, 32, 1e2)
    b = si.rhs_uniform(64, 64, 32, 1001)
    o = pcg.pcg_default_opts(precision=pcg.PCG_PREC_MIXED, preconditioner=MG)
    arena = torch.empty(pcg.pcg_request_bytes(d, o) + (1 << 20), dtype=torch.uint8, device="cuda")
    srv = pcg.Server(arena, arena.numel(), 1)
    try:
        xh = np.zeros_like(b)
        t = pcg.pcg_submit(srv, d, b, xh, o)
        st, r = pcg.pcg_wait(srv, t)
        assert st == pcg.PCG_OK, r
    finally:
        srv.close()
    p = pcg.Problem(d)
    o.x0_zero = 1
    bt = cuda(b)
    x = torch.zeros_like(bt)
    st, _ = pcg.pcg_solve(p, bt, x, pcg.workspace(p, o), o)
    assert st == pcg.PCG_OK
    np.testing.assert_array_equal(x.cpu().numpy(), xh)


def test_full_size_weak_anisotropy_mg():
    """512 x 512 x 128 Dirichlet with anisotropy 1e2 (the regime where line
    relaxation alone needs many iterations): MG-PCG converges with the
    oracle's assembled matrix checking the residual."""
    d = desc(512, 512, 128, 1e2)
    p = pcg.Problem(d)
    b = si.rhs_uniform(512, 512, 128, 1)
    x, st, res = gpu_solve(p, b, true_residual=1)
    assert st == pcg.PCG_OK
    A = oracle.assemble(grid_of(d, None, None))
    true = oracle.residual_norm(A, b, x) / np.linalg.norm(b)
    print("MG 512x512x128 1e2: %d iterations, true residual %.3e" % (res["iterations"], true))
    assert true < 1.05e-8
