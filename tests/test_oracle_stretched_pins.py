"""Pins for the oracle on stretched (non-uniform tensor-product) horizontal
grids, against facts that do not come from the oracle's own assembly loop.

* Kronecker structure: on a tensor-product grid the finite-volume operator is
  M_x(x)M_y(x)M_z + K_h (S_x(x)M_y(x)M_z + M_x(x)S_y(x)M_z) + K_v M_x(x)M_y(x)S_z,
  with M = diag(widths) and S the 1D two-point-flux stiffness (face weight
  1 / distance between centres, 2 / width at a Dirichlet face, wrap-around
  for periodic sides).  Built here from 1D matrices and compared entry by
  entry: pins every area, distance, Dirichlet factor and periodic seam.
* Separable eigenpairs: Kronecker products of the 1D generalised
  eigenvectors (S v = lambda M v, from LAPACK) are eigenvectors of A in the
  form A v = [1 + K_h (lx + ly) + K_v lz] (M v).
* Linear exactness: the two-point flux through a face is exact for a field
  linear in the normal coordinate when the distance is the one between cell
  centres, so A u = V u in rows whose faces all see the linear field (and
  the Dirichlet half-cell factor is exact for a field vanishing on the wall).
* Symmetry, definiteness, dense direct solves and the K_h = 0 one-step case
  carry over from the uniform grid.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import synth_inputs as si


def stretched_grids():
    return [
        oracle.Grid(5, 4, 6, 0, 0, 1.0, 1.05, 1.0, 40.0, False, False,
                    tuple(si.widths_random(5, 11)), tuple(si.widths_graded(4, 1.3))),
        oracle.Grid(6, 5, 4, 0, 0, 2.0, 1.2, 0.7, 3.0, True, False,
                    tuple(si.widths_sine(6, 0.6)), tuple(si.widths_random(5, 12, 0.2, 2.0))),
        oracle.Grid(4, 7, 5, 0, 0, 1.0, 1.0, 1.3, 500.0, True, True,
                    tuple(si.widths_random(4, 13)), tuple(si.widths_sine(7, 0.4, 2.0))),
        oracle.Grid(3, 3, 8, 0, 0, 1.0, 1.1, 1.0, 1e4, False, True,
                    tuple(si.widths_graded(3, 2.0, 0.5)), tuple(si.widths_random(3, 14))),
    ]


IDS = lambda g: f"{g.nx}x{g.ny}x{g.nz}p{int(g.per_x)}{int(g.per_y)}"


def dense(A):
    return A.to_scipy().toarray()


def stiffness_1d(w, periodic):
    """1D two-point-flux stiffness on cells of widths w."""
    n = w.size
    S = np.zeros((n, n))
    for i in range(n - 1):
        t = 1.0 / (0.5 * (w[i] + w[i + 1]))
        S[i, i] += t
        S[i + 1, i + 1] += t
        S[i, i + 1] -= t
        S[i + 1, i] -= t
    if periodic:
        t = 1.0 / (0.5 * (w[0] + w[-1]))
        S[0, 0] += t
        S[-1, -1] += t
        S[0, -1] -= t
        S[-1, 0] -= t
    else:
        S[0, 0] += 2.0 / w[0]
        S[-1, -1] += 2.0 / w[-1]
    return S


def factors(g):
    xw, yw = g.widths()
    dz = oracle.vertical_spacing(g.nz, g.H, g.q)
    return ((np.diag(xw), stiffness_1d(xw, g.per_x)), (np.diag(yw), stiffness_1d(yw, g.per_y)),
            (np.diag(dz), stiffness_1d(dz, False)))


@pytest.mark.parametrize("g", stretched_grids(), ids=IDS)
def test_operator_has_the_tensor_product_structure(g):
    (Mx, Sx), (My, Sy), (Mz, Sz) = factors(g)
    K = np.kron
    want = (K(K(Mx, My), Mz) + g.kh * (K(K(Sx, My), Mz) + K(K(Mx, Sy), Mz))
            + g.kv * K(K(Mx, My), Sz))
    got = dense(oracle.assemble(g))
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-13 * np.abs(want).max())
    assert np.array_equal(got != 0, np.abs(want) > 1e-13 * np.abs(want).max())


@pytest.mark.parametrize("g", stretched_grids(), ids=IDS)
def test_separable_generalised_eigenpairs(g):
    (Mx, Sx), (My, Sy), (Mz, Sz) = factors(g)
    lx, Vx = sla.eigh(Sx, Mx)
    ly, Vy = sla.eigh(Sy, My)
    lz, Vz = sla.eigh(Sz, Mz)
    A = oracle.assemble(g)
    rng = np.random.default_rng(21)
    for _ in range(6):
        a, b, c = rng.integers(g.nx), rng.integers(g.ny), rng.integers(g.nz)
        v = np.kron(np.kron(Vx[:, a], Vy[:, b]), Vz[:, c])
        mv = np.kron(np.kron(Mx @ Vx[:, a], My @ Vy[:, b]), Mz @ Vz[:, c])
        mu = 1.0 + g.kh * (lx[a] + ly[b]) + g.kv * lz[c]
        Av = A.matvec(v)
        np.testing.assert_allclose(Av, mu * mv, rtol=0, atol=1e-11 * np.abs(Av).max())


def test_linear_fields_reproduced_exactly():
    # Dirichlet in x (wall at x = 0), periodic in y, u = x-coordinate of the
    # cell centre: zero net flux in every cell except the last x-column
    # (whose wall sees u != 0) and the top/bottom levels (Dirichlet in z).
    xw = si.widths_random(7, 31, 0.3, 3.0)
    yw = si.widths_random(5, 32)
    g = oracle.Grid(7, 5, 6, 0, 0, 1.0, 1.07, 0.9, 15.0, False, True, tuple(xw), tuple(yw))
    xc = np.cumsum(xw) - 0.5 * xw
    u = np.broadcast_to(xc[:, None, None], (g.nx, g.ny, g.nz)).ravel().copy()
    dz = oracle.vertical_spacing(g.nz, g.H, g.q)
    vol = (xw[:, None, None] * yw[None, :, None] * dz[None, None, :]).ravel()
    r = (oracle.assemble(g).matvec(u) - vol * u).reshape(g.nx, g.ny, g.nz)
    inner = r[:-1, :, 1:-1]
    assert np.abs(inner).max() <= 1e-13 * np.abs(vol * u).max() * 100
    assert np.abs(r[-1, :, 1:-1]).min() > 1e-3        # the far wall does see the field
    # the same in y with u = y-coordinate, periodic x, Dirichlet y
    g = oracle.Grid(5, 7, 6, 0, 0, 1.0, 1.07, 0.9, 15.0, True, False, tuple(yw), tuple(xw))
    u = np.broadcast_to(xc[None, :, None], (g.nx, g.ny, g.nz)).ravel().copy()
    vol = (yw[:, None, None] * xw[None, :, None] * dz[None, None, :]).ravel()
    r = (oracle.assemble(g).matvec(u) - vol * u).reshape(g.nx, g.ny, g.nz)
    assert np.abs(r[:, :-1, 1:-1]).max() <= 1e-13 * np.abs(vol * u).max() * 100


@pytest.mark.parametrize("g", stretched_grids(), ids=IDS)
def test_symmetric_dominant_definite(g):
    D = dense(oracle.assemble(g))
    assert np.array_equal(D, D.T)
    diag = np.diag(D)
    off = np.abs(D).sum(axis=1) - np.abs(diag)
    assert np.all(diag - off > 0)
    assert np.linalg.eigvalsh(D).min() > 0


@pytest.mark.parametrize("g", stretched_grids(), ids=IDS)
def test_pcg_and_line_solve_match_dense_solves(g):
    A = oracle.assemble(g)
    M = oracle.line_blocks(A, g.nz)
    Md = np.diag(M.di) + np.diag(M.lo[1:], -1) + np.diag(M.up[:-1], 1)
    r = np.random.default_rng(5).standard_normal(g.n)
    zd = np.linalg.solve(Md, r)
    np.testing.assert_allclose(oracle.line_solve(M, r), zd, rtol=1e-13,
                               atol=1e-13 * np.abs(zd).max())
    b = si.rhs_uniform(g.nx, g.ny, g.nz, 0)
    res = oracle.pcg(A, M, b, rtol=1e-14)
    xd = sla.cho_solve(sla.cho_factor(dense(A)), b)
    assert res["status"] == "converged"
    assert np.linalg.norm(res["x"] - xd) <= 1e-12 * np.linalg.norm(xd)


def test_no_horizontal_coupling_one_iteration_on_stretched_grid():
    g = oracle.Grid(6, 5, 16, 0, 0, 1.0, 1.05, 0.0, 1e3, False, False,
                    tuple(si.widths_random(6, 41)), tuple(si.widths_sine(5)))
    A = oracle.assemble(g)
    res = oracle.pcg(A, oracle.line_blocks(A, g.nz), si.rhs_uniform(6, 5, 16, 3), rtol=1e-12)
    assert res["status"] == "converged" and res["iterations"] == 1


def test_row_apply_matches_assembled_rows_on_stretched_grids():
    rng = np.random.default_rng(17)
    for g in stretched_grids():
        A = oracle.assemble(g)
        x = rng.standard_normal(g.n)
        y = A.matvec(x).reshape(g.nx, g.ny, g.nz)
        for _ in range(10):
            i, j, k = rng.integers(g.nx), rng.integers(g.ny), rng.integers(g.nz)
            assert oracle.row_apply(g, i, j, k, x) == pytest.approx(y[i, j, k], rel=1e-14, abs=1e-14)


def test_width_recipes():
    for w in (si.widths_sine(64), si.widths_graded(50, 1.1, 2.0), si.widths_random(33, 5)):
        assert np.all(w > 0)
    assert abs(si.widths_sine(64).sum() - 1.0) < 1e-14
    assert abs(si.widths_graded(50, 1.1, 2.0).sum() - 2.0) < 1e-14
    w = si.widths_sine(64, 0.5)
    assert 2.9 < w.max() / w.min() < 3.0
