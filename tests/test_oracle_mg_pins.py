"""Pins for the oracle's tensor-product multigrid preconditioner
(oracle/mg.py) against facts that do not come from its own code:

* intergrid operators: restriction is exactly the transpose of the
  prolongation, conserves the total residual, and the prolongation keeps
  constants;
* coarse operators: on a periodic grid a field that is constant in the
  horizontal sees the same operator on the coarse grid as the Galerkin
  product P^T A P (mass and vertical terms scale with the merged area);
* one level: the V-cycle is k damped line-Jacobi sweeps from zero, i.e.
  (I - (I - omega M^{-1} A)^k) A^{-1} (closed form with dense matrices);
* the V-cycle is a symmetric positive definite operator (so CG applies);
* with the vertical coupling fixed while the horizontal grid is refined,
  the line preconditioner's condition number grows like h^-2 while the
  V-cycle's stays small (growing mildly with the number of levels), and
  MG-preconditioned CG needs a bounded number of iterations (the reason
  multigrid is named as the next step);
* the MG-preconditioned CG solution matches a dense direct solve.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import oracle.mg as mg
import synth_inputs as si


def dense(A):
    return A.to_scipy().toarray()


def dense_op(f, n):
    return np.stack([f(e) for e in np.eye(n)], axis=1)


def test_level_sequence():
    g = oracle.grid_from_ratio(64, 32, 8, 1e3)
    assert [(x.nx, x.ny) for x in mg.levels(g)] == [(64, 32), (32, 16), (16, 8), (8, 4)]
    assert [(x.nx, x.ny) for x in mg.levels(g, 2)] == [(64, 32), (32, 16)]
    assert len(mg.levels(oracle.grid_from_ratio(12, 10, 4, 1e3))) == 2     # 10 -> 5 (odd)
    assert len(mg.levels(oracle.grid_from_ratio(7, 8, 4, 1e3))) == 1
    c = mg.coarse_grid(g)
    assert (c.dx, c.dy, c.nz, c.kv) == (2 * g.dx, 2 * g.dy, g.nz, g.kv)
    gs = oracle.Grid(8, 8, 3, 0, 0, 1.0, 1.05, 1.0, 10.0, False, True,
                     tuple(si.widths_random(8, 1)), tuple(si.widths_sine(8)))
    cs = mg.coarse_grid(gs)
    np.testing.assert_allclose(cs.widths()[0], si.widths_random(8, 1).reshape(4, 2).sum(1))


@pytest.mark.parametrize("per", [False, True])
def test_restriction_is_the_transpose_of_prolongation(per):
    gf = oracle.grid_from_ratio(8, 12, 5, 1e3, periodic=per)
    gc = mg.coarse_grid(gf)
    rng = np.random.default_rng(3)
    r, zc = rng.standard_normal(gf.n), rng.standard_normal(gc.n)
    a, b = mg.restrict(gf, gc, r) @ zc, r @ mg.prolong(gf, gc, zc)
    assert abs(a - b) <= 1e-13 * np.abs(r).sum() * np.abs(zc).max()
    assert abs(mg.restrict(gf, gc, r).sum() - r.sum()) <= 1e-12 * np.abs(r).sum()
    assert np.all(mg.prolong(gf, gc, np.full(gc.n, 2.5)) == 2.5)
    # every fine column's parent is the coarse column containing it
    P = dense_op(lambda v: mg.prolong(gf, gc, v), gc.n)
    assert np.all(P.sum(axis=1) == 1) and np.all(P.sum(axis=0) == 4)


@pytest.mark.parametrize("stretched", [False, True])
def test_coarse_operator_on_horizontally_constant_fields(stretched):
    if stretched:
        gf = oracle.Grid(8, 12, 6, 0, 0, 1.0, 1.1, 0.7, 30.0, True, True,
                         tuple(si.widths_random(8, 4)), tuple(si.widths_sine(12)))
    else:
        gf = oracle.grid_from_ratio(8, 12, 6, 1e3, periodic=True)
    gc = mg.coarse_grid(gf)
    Af, Ac = oracle.assemble(gf), oracle.assemble(gc)
    f = np.random.default_rng(5).standard_normal(gf.nz)
    vc = np.tile(f, gc.nx * gc.ny)
    galerkin = mg.restrict(gf, gc, Af.matvec(mg.prolong(gf, gc, vc)))
    np.testing.assert_allclose(Ac.matvec(vc), galerkin, rtol=1e-12, atol=1e-12 * np.abs(galerkin).max())


def test_single_level_is_damped_line_jacobi_closed_form():
    g = oracle.grid_from_ratio(5, 4, 6, 1e2)
    h = mg.Hierarchy(g)
    assert len(h.grids) == 1
    A = dense(h.A[0])
    M = h.M[0]
    Md = np.diag(M.di) + np.diag(M.lo[1:], -1) + np.diag(M.up[:-1], 1)
    E = np.eye(g.n) - mg.OMEGA * np.linalg.solve(Md, A)
    want = (np.eye(g.n) - np.linalg.matrix_power(E, mg.COARSE_SWEEPS)) @ np.linalg.inv(A)
    got = dense_op(h.vcycle, g.n)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-10 * np.abs(want).max())


@pytest.mark.parametrize("args", [(16, 8, 4, 1e1, False), (8, 8, 5, 1e3, True), (16, 16, 3, 1e2, False)])
def test_vcycle_is_symmetric_positive_definite(args):
    nx, ny, nz, g2, per = args
    g = oracle.grid_from_ratio(nx, ny, nz, g2, periodic=per)
    h = mg.Hierarchy(g)
    assert len(h.grids) >= 2
    B = dense_op(h.vcycle, g.n)
    assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0


def _kappa(B, A):
    ev = np.linalg.eigvals(B @ A).real
    return ev.max() / ev.min()


def _fixed_kv_grid(n, nz):
    # fixed K_v while the horizontal grid is refined: the vertical coupling
    # weakens relative to the horizontal one, so the line preconditioner's
    # condition number grows like n^2 while multigrid's stays bounded
    return oracle.Grid(n, n, nz, 1.0 / n, 1.0 / n, 1.0, 1.05, 1.0, 0.05, False, False)


def test_condition_number_small_and_grid_independent():
    kap_mg, kap_line = [], []
    for n in (8, 16, 32):
        g = _fixed_kv_grid(n, 4)
        h = mg.Hierarchy(g)
        A = dense(h.A[0])
        B = dense_op(h.vcycle, g.n)
        M = h.M[0]
        Md = np.diag(M.di) + np.diag(M.lo[1:], -1) + np.diag(M.up[:-1], 1)
        kap_mg.append(_kappa(B, A))
        kap_line.append(sla.eigh(A, Md, eigvals_only=True)[[0, -1]])
    kap_line = [e[1] / e[0] for e in kap_line]
    # line relaxation alone: kappa ~ h^-2 (x4 per refinement); the V-cycle:
    # small, growing only mildly with the number of levels (one per
    # refinement; piecewise-constant prolongation)
    assert max(kap_mg) < 4.0, kap_mg
    assert all(kap_mg[i + 1] < 1.3 * kap_mg[i] for i in range(2)), kap_mg
    assert all(kap_line[i + 1] > 3.5 * kap_line[i] for i in range(2)), kap_line
    assert kap_line[2] > 50 * kap_mg[2], (kap_line, kap_mg)


def test_iterations_bounded_independent_of_grid_size():
    its = []
    for n in (16, 32, 64, 128):
        g = _fixed_kv_grid(n, 16)
        res = mg.solve(g, si.rhs_uniform(n, n, 16, 0))
        assert res["status"] == "converged"
        its.append(res["iterations"])
    line = oracle.solve(_fixed_kv_grid(128, 16), si.rhs_uniform(128, 128, 16, 0))
    # a few more iterations per added level (piecewise-constant prolongation);
    # the line preconditioner alone needs ~2x more per refinement
    assert all(its[i + 1] - its[i] <= 3 for i in range(3)) and max(its) <= 22, its
    assert line["iterations"] > 4 * max(its), (line["iterations"], its)


@pytest.mark.parametrize("args", [(16, 8, 6, 1e2, False, 0), (8, 8, 5, 1e4, True, 0),
                                  (16, 16, 4, 1e1, False, 2)])
def test_mg_pcg_matches_dense_solve(args):
    nx, ny, nz, g2, per, ml = args
    g = oracle.grid_from_ratio(nx, ny, nz, g2, periodic=per)
    b = si.rhs_uniform(nx, ny, nz, 7)
    res = mg.solve(g, b, rtol=1e-13, max_levels=ml)
    assert res["status"] == "converged"
    xd = np.linalg.solve(dense(res["A"]), b)
    assert np.linalg.norm(res["x"] - xd) <= 1e-11 * np.linalg.norm(xd)


def test_stretched_grid_multigrid_converges():
    g = oracle.Grid(32, 32, 16, 0, 0, 1.0, 1.05, 1.0, 0.5, False, False,
                    tuple(si.widths_sine(32, 0.5)), tuple(si.widths_graded(32, 1.05)))
    res = mg.solve(g, si.rhs_uniform(32, 32, 16, 0))
    line = oracle.solve(g, si.rhs_uniform(32, 32, 16, 0))
    assert res["status"] == "converged" and res["iterations"] * 3 < line["iterations"]
