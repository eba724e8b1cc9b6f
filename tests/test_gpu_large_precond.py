"""Multigrid and block Gauss-Seidel at a size where their kernels stream the
fine level with the nontemporal hint (vectors of 64 MiB: 256 x 256 x 128
FP64) and run one column per wavefront (64 lanes per column for every
kernel), against the oracle, through the C ABI.

* one V-cycle and one block Gauss-Seidel application equal the oracle's
  (the V-cycle's coarser levels take the plain loads: the test covers both);
* three FP64 iterations of MG-PCG and of RBGS-PCG equal the oracle's
  iterates (the fused first and last kernels of each preconditioner phase).
Tolerances as for the small grids (per column: no column's error may
exceed them): the same linear maps computed in another order."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
import oracle.mg as omg  # noqa: E402
import oracle.rbgs as rb  # noqa: E402
import paper_1302_7193_amd as pcg  # noqa: E402
import synth_inputs as si  # noqa: E402
from _checks import column_rel_errors  # noqa: E402

NX, NY, NZ = 256, 256, 128


@pytest.fixture(scope="module")
def case():
    d = pcg.pcg_desc_from_ratio(NX, NY, NZ, 1.05, 1e2, pcg.PCG_BC_DIRICHLET)
    assert d.nx * d.ny * d.nz * 8 >= 64 << 20
    g = oracle.Grid(d.nx, d.ny, d.nz, d.dx, d.dy, d.height, d.grading, d.k_h, d.k_v,
                    False, False)
    p = pcg.Problem(d)
    pcg.pcg_set_tuning(p, pcg.PCG_F64, lanes_per_column=64, lanes_per_column_prec=64)
    t = pcg.pcg_get_tuning(p, pcg.PCG_F64)
    assert t.lanes_per_column == 64 and t.lanes_per_column_prec == 64
    A = oracle.assemble(g)
    return d, g, p, A


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_vcycle_and_rbgs_match_oracle(case):
    d, g, p, A = case
    print("large vcycle / rbgs", NX, NY, NZ, flush=True)
    r = si.uniform_pm1(71, p.n)
    rt = cuda(r)
    z = torch.full_like(rt, float("nan"))
    levels = pcg.pcg_mg_levels(p)
    ws = torch.empty(pcg.pcg_mg_bytes(p, pcg.PCG_F64, levels), dtype=torch.uint8, device="cuda")
    pcg.pcg_mg_precond(p, pcg.PCG_F64, rt, z, ws, levels)
    torch.cuda.synchronize()
    want = omg.Hierarchy(g).vcycle(r)
    err = column_rel_errors(z.cpu().numpy(), want, NZ).max()
    print("large vcycle: worst column error %.2e" % err)
    assert err <= 1e-11, err
    z.fill_(float("nan"))
    pcg.pcg_rbgs_precond(p, pcg.PCG_F64, rt, z)
    torch.cuda.synchronize()
    want = rb.RBGS(g, A).apply(r)
    err = column_rel_errors(z.cpu().numpy(), want, NZ).max()
    print("large rbgs: worst column error %.2e" % err)
    assert err <= 1e-11, err


@pytest.mark.parametrize("prec", [pcg.PCG_PRECOND_MG, pcg.PCG_PRECOND_RBGS])
def test_fp64_pcg_equal_iterations(case, prec):
    d, g, p, A = case
    print("large solve", prec, flush=True)
    b = si.rhs_uniform(NX, NY, NZ, 5)
    k = 3
    apply = omg.Hierarchy(g).vcycle if prec == pcg.PCG_PRECOND_MG else rb.RBGS(g, A).apply
    ref = omg.pcg(A, apply, b, rtol=0.0, max_iter=k)
    assert ref["iterations"] == k
    o = pcg.pcg_default_opts(preconditioner=prec, rtol=0.0, max_iter=k)
    bt = cuda(b)
    x = torch.zeros_like(bt)
    st, res = pcg.pcg_solve(p, bt, x, pcg.workspace(p, o), o)
    assert res["iterations"] == k and res["preconditioner"] == prec
    xs = x.cpu().numpy()
    err = np.linalg.norm(xs - ref["x"]) / np.linalg.norm(ref["x"])
    assert err <= 1e-10, err
