"""Pins for the oracle's symmetric red-black block Gauss-Seidel
preconditioner (oracle/rbgs.py):

* it is the textbook symmetric Gauss-Seidel operator: with the columns in
  red-black order, M = (D + L) D^{-1} (D + U) for the column blocks D and the
  strictly lower / upper block parts L, U of A (dense matrices; pins the
  sweep order and the couplings used in each half-sweep);
* symmetric positive definite; exact (one CG iteration) when there are no
  couplings between columns; roughly halves line relaxation's iterations;
* PCG with it matches a dense direct solve."""
import numpy as np
import pytest

import oracle
import oracle.mg as omg
import oracle.rbgs as rb
import synth_inputs as si


def dense(A):
    return A.to_scipy().toarray()


GRIDS = [
    oracle.grid_from_ratio(4, 5, 4, 1e2),
    oracle.grid_from_ratio(6, 4, 5, 1e1, periodic=True),
    oracle.Grid(5, 4, 3, 0.3, 0.2, 1.0, 1.2, 0.8, 2.0, False, True),
    oracle.Grid(4, 6, 4, 0, 0, 1.0, 1.05, 1.0, 5.0, True, False,
                tuple(si.widths_random(4, 3)), tuple(si.widths_sine(6))),
]
IDS = lambda g: f"{g.nx}x{g.ny}x{g.nz}p{int(g.per_x)}{int(g.per_y)}"


@pytest.mark.parametrize("g", GRIDS, ids=IDS)
def test_equals_textbook_symmetric_gauss_seidel(g):
    A = dense(oracle.assemble(g))
    red = rb.red_mask(g)
    order = np.concatenate([np.flatnonzero(red), np.flatnonzero(~red)])
    Ap = A[np.ix_(order, order)]
    col = (order // g.nz)
    same = col[:, None] == col[None, :]
    D = np.where(same, Ap, 0.0)
    L = np.tril(Ap - D)
    U = np.triu(Ap - D)
    Mp = (D + L) @ np.linalg.solve(D, D + U)
    p = rb.RBGS(g)
    rng = np.random.default_rng(1)
    for _ in range(3):
        r = rng.standard_normal(g.n)
        want = np.empty(g.n)
        want[order] = np.linalg.solve(Mp, r[order])
        np.testing.assert_allclose(p.apply(r), want, rtol=0, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("g", GRIDS, ids=IDS)
def test_symmetric_positive_definite(g):
    p = rb.RBGS(g)
    B = np.stack([p.apply(e) for e in np.eye(g.n)], axis=1)
    assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0


def test_exact_without_horizontal_coupling():
    g = oracle.Grid(6, 4, 8, 1 / 6, 1 / 4, 1.0, 1.05, 0.0, 1e2, False, False)
    A = oracle.assemble(g)
    res = omg.pcg(A, rb.RBGS(g, A).apply, si.rhs_uniform(6, 4, 8, 2), rtol=1e-12)
    assert res["status"] == "converged" and res["iterations"] == 1


def test_halves_line_relaxation_iterations():
    for args in ((32, 32, 32, 1e2), (32, 32, 64, 1e1)):
        g = oracle.grid_from_ratio(*args)
        A = oracle.assemble(g)
        b = si.rhs_uniform(g.nx, g.ny, g.nz, 0)
        line = oracle.pcg(A, oracle.line_blocks(A, g.nz), b)["iterations"]
        its = omg.pcg(A, rb.RBGS(g, A).apply, b)["iterations"]
        assert its <= 0.6 * line, (its, line)


@pytest.mark.parametrize("g", GRIDS, ids=IDS)
def test_pcg_matches_dense_solve(g):
    A = oracle.assemble(g)
    b = si.rhs_uniform(g.nx, g.ny, g.nz, 5)
    res = omg.pcg(A, rb.RBGS(g, A).apply, b, rtol=1e-13)
    xd = np.linalg.solve(dense(A), b)
    assert res["status"] == "converged"
    assert np.linalg.norm(res["x"] - xd) <= 1e-11 * np.linalg.norm(xd)


def test_odd_periodic_rejected():
    with pytest.raises(ValueError):
        rb.RBGS(oracle.grid_from_ratio(5, 4, 3, 1e2, periodic=True))
