"""Allocation-free solve (pcg_solve_noalloc) through the C ABI against
pcg_solve with a caller workspace: two calls in a row, the second on a
smaller grid, in FP64 (zero and non-zero start) and mixed precision, must
give bitwise the same solution and result as pcg_solve (the same kernels
and launch parameters; direct launches equal graph chunks bitwise), and
the FP64 one the oracle's iterate at an equal iteration count to 1e-10.  A
solve whose workspace exceeds the fixed scratch is rejected."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_1302_7193_amd as pcg  # noqa: E402
import synth_inputs as si  # noqa: E402


def grid(nx, ny, nz, g2):
    d = pcg.pcg_desc_from_ratio(nx, ny, nz, 1.05, g2, pcg.PCG_BC_DIRICHLET)
    g = oracle.Grid(d.nx, d.ny, d.nz, d.dx, d.dy, d.height, d.grading, d.k_h, d.k_v,
                    False, False)
    return d, g


@pytest.mark.parametrize("precision,x0_zero", [(pcg.PCG_PREC_FP64, 1), (pcg.PCG_PREC_FP64, 0),
                                               (pcg.PCG_PREC_MIXED, 1)])
def test_noalloc_equals_pcg_solve_on_two_calls(precision, x0_zero):
    for call, (nx, ny, nz, g2, seed) in enumerate(((64, 64, 32, 1e4, 0), (13, 7, 33, 1e3, 3))):
        print("noalloc call %d: %dx%dx%d precision %d x0_zero %d" % (call, nx, ny, nz, precision,
                                                                    x0_zero), flush=True)
        d, g = grid(nx, ny, nz, g2)
        p = pcg.Problem(d)
        b = si.rhs_uniform(nx, ny, nz, seed)
        x0 = 0.01 * si.uniform_pm1(seed + 50, p.n) if not x0_zero else np.zeros(p.n)
        A = oracle.assemble(g)
        M = oracle.line_blocks(A, nz)
        kw = dict(precision=precision, x0_zero=x0_zero)
        if precision == pcg.PCG_PREC_FP64:
            k = oracle.pcg(A, M, b, x0=x0, rtol=1e-8)["iterations"]
            kw.update(rtol=0.0, max_iter=k)
        o = pcg.pcg_default_opts(**kw)
        bt = torch.from_numpy(b).cuda()
        xw = torch.from_numpy(x0).cuda() if not x0_zero else torch.full_like(bt, float("nan"))
        st_w, r_w = pcg.pcg_solve(p, bt, xw, pcg.workspace(p, o), o)
        xn = torch.from_numpy(x0).cuda() if not x0_zero else torch.full_like(bt, float("nan"))
        st_n, r_n = pcg.pcg_solve_noalloc(p, bt, xn, o)
        assert st_n == st_w
        assert r_n["iterations"] == r_w["iterations"] and r_n["status"] == r_w["status"]
        assert r_n["rel_res_recursive"] == r_w["rel_res_recursive"]
        xs = xn.cpu().numpy()
        assert np.array_equal(xs, xw.cpu().numpy())
        if precision == pcg.PCG_PREC_FP64:
            ref = oracle.pcg(A, M, b, x0=x0, rtol=0.0, max_iter=k)
            err = np.linalg.norm(xs - ref["x"]) / np.linalg.norm(ref["x"])
            assert r_n["iterations"] == k and err <= 1e-10, err
        else:
            assert st_n == pcg.PCG_OK
            assert oracle.residual_norm(A, b, xs) / np.linalg.norm(b) < 1e-8


def test_noalloc_rejects_a_solve_larger_than_its_scratch():
    d, _ = grid(256, 256, 128, 1e3)
    p = pcg.Problem(d)
    bt = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    xt = torch.empty_like(bt)
    with pytest.raises(pcg.PCGError) as e:
        pcg.pcg_solve_noalloc(p, bt, xt)
    assert e.value.status == pcg.PCG_E_NOMEM
    assert "scratch" in pcg.pcg_last_error()
