"""Pins for the CPU oracle against facts fixed by the paper and by mathematics,
not by the oracle itself.

Each test names what it pins.  A plausible slip anywhere in the oracle (a
dropped face term, a wrong sign, a missing half-cell factor at a Dirichlet
face, a transposed index, a wrong Thomas recurrence, an off-by-one in the CG
loop) fails at least one of them:

* symmetry / definiteness / conservation    -> signs and pairing of face terms
* closed-form eigenpairs (uniform grid)     -> every transmissibility and the
                                               Dirichlet half-cell factor
* manufactured-solution convergence order   -> the graded vertical spacing and
                                               the operator as a whole
* dense direct solves, n_z = 1 Jacobi,
  single column M == A                      -> preconditioner and Thomas solve
* K_h = 0 one-step convergence, dense
  Cholesky, CG orthogonality / error bound,
  interleaved (Alg. InterleavedPCG) equal
  to standard PCG                           -> the Krylov loop
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import synth_inputs as si

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense(A):
    return A.to_scipy().toarray()


def small_grids():
    return [
        oracle.grid_from_ratio(3, 3, 4, 1e2, q=1.05, periodic=False),
        oracle.grid_from_ratio(4, 5, 6, 1e3, q=1.05, periodic=False),
        oracle.grid_from_ratio(3, 4, 5, 1e2, q=1.05, periodic=True),
        oracle.grid_from_ratio(5, 3, 7, 1e4, q=1.10, periodic=True),
        oracle.Grid(4, 3, 5, 0.3, 0.2, 2.0, 1.2, 0.7, 3.0, True, False),
    ]


# --------------------------------------------------------------- grid ---

def test_vertical_spacing_geometric_and_sums_to_height():
    for nz, H, q in [(32, 1.0, 1.05), (7, 2.5, 1.3), (128, 1.0, 1.05)]:
        dz = oracle.vertical_spacing(nz, H, q)
        assert abs(dz.sum() - H) <= 1e-13 * H
        np.testing.assert_allclose(dz[1:] / dz[:-1], q, rtol=1e-13)
        assert dz.argmin() == 0            # finest cell at the ground
    dz = oracle.vertical_spacing(16, 3.0, 1.0)
    np.testing.assert_allclose(dz, 3.0 / 16, rtol=0, atol=1e-15)


def test_kv_from_ratio_closed_form_values():
    # gamma^2 = (K_v / (H/n_z)^2) / (K_h / dx^2) with K_h = 1, H = 1, dx = 1/n_x
    # => K_v = gamma^2 (n_x / n_z)^2 for the five workload shapes.
    cases = [((64, 32, 1e4), 4e4), ((512, 128, 1e5), 1.6e6),
             ((1024, 128, 1e4), 6.4e5), ((256, 64, 1e3), 1.6e4)]
    for (nx, nz, g2), kv in cases:
        g = oracle.grid_from_ratio(nx, nx, nz, g2)
        assert abs(g.kv - kv) <= 1e-12 * kv


# ----------------------------------------------------------- assembly ---

@pytest.mark.parametrize("g", small_grids(), ids=lambda g: f"{g.nx}x{g.ny}x{g.nz}p{int(g.per_x)}{int(g.per_y)}")
def test_assembled_matrix_exactly_symmetric(g):
    D = dense(oracle.assemble(g))
    assert np.array_equal(D, D.T)


@pytest.mark.parametrize("g", small_grids(), ids=lambda g: f"{g.nx}x{g.ny}x{g.nz}")
def test_bilinear_form_symmetry_random_vectors(g):
    A = oracle.assemble(g)
    rng = np.random.default_rng(7)
    for _ in range(5):
        x, y = rng.standard_normal(g.n), rng.standard_normal(g.n)
        a, b = x @ A.matvec(y), y @ A.matvec(x)
        assert abs(a - b) <= 1e-14 * (abs(a) + np.abs(x) @ np.abs(dense(A)) @ np.abs(y))


@pytest.mark.parametrize("g", small_grids(), ids=lambda g: f"{g.nx}x{g.ny}x{g.nz}")
def test_strict_diagonal_dominance_and_positive_definite(g):
    D = dense(oracle.assemble(g))
    dz = oracle.vertical_spacing(g.nz, g.H, g.q)
    vol = np.tile(g.dx * g.dy * dz, g.nx * g.ny)
    diag = np.diag(D)
    off = np.abs(D).sum(axis=1) - np.abs(diag)
    assert np.all(diag > 0)
    # diag - sum|off| = V + (Dirichlet face terms) >= V  (Gershgorin => SPD)
    # (the difference cancels to ~V << diag: allow rounding relative to diag)
    assert np.all(diag - off >= vol - 1e-13 * diag)
    ev = np.linalg.eigvalsh(D)
    assert ev.min() >= vol.min() * (1 - 1e-10)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((g.n, 8))
    assert np.all(np.einsum("ij,ij->j", x, D @ x) > 0)


def test_conservation_row_sums():
    # A constant field has zero flux through every interior or periodic face,
    # so a row sum equals the cell volume unless the cell touches a Dirichlet
    # face; there it is larger by the boundary transmissibility
    # 2*K*area/spacing (half-cell distance).
    g = oracle.Grid(5, 4, 6, 0.25, 0.5, 1.5, 1.1, 0.8, 20.0, False, True)
    A = oracle.assemble(g)
    s = A.matvec(np.ones(g.n)).reshape(g.nx, g.ny, g.nz)
    dz = oracle.vertical_spacing(g.nz, g.H, g.q)
    vol = g.dx * g.dy * dz
    expect = np.broadcast_to(vol, (g.nx, g.ny, g.nz)).copy()
    xface = 2 * g.kh * g.dy * dz / g.dx
    expect[0] += xface
    expect[-1] += xface
    expect[:, :, 0] += 2 * g.kv * g.dx * g.dy / dz[0]
    expect[:, :, -1] += 2 * g.kv * g.dx * g.dy / dz[-1]
    np.testing.assert_allclose(s, expect, rtol=1e-12, atol=1e-14)


def _mode(n, m, periodic):
    i = np.arange(n)
    if periodic:
        return np.cos(2 * np.pi * m * i / n), 4 * np.sin(np.pi * m / n) ** 2
    return np.sin(np.pi * m * (i + 0.5) / n), 4 * np.sin(np.pi * m / (2 * n)) ** 2


@pytest.mark.parametrize("per", [False, True])
def test_closed_form_eigenpairs_uniform_grid(per):
    # q = 1: the operator is a Kronecker sum of 1-D second differences
    # (Dirichlet: ghost = -u, eigvec sin(pi m (i+1/2)/n), eigval 4 sin^2(pi m/2n);
    #  periodic: cos(2 pi m i/n), eigval 4 sin^2(pi m/n)), so a product mode
    # v satisfies A v = V (1 + K_h lx/dx^2 + K_h ly/dy^2 + K_v lz/dz^2) v.
    g = oracle.Grid(6, 5, 8, 0.3, 0.45, 2.0, 1.0, 1.7, 55.0, per, per)
    A = oracle.assemble(g)
    dzu = g.H / g.nz
    V = g.dx * g.dy * dzu
    for mx, my, mz in [(1, 1, 1), (2, 3, 5), (5, 4, 8), (3, 1, 2)]:
        vx, lx = _mode(g.nx, mx, per)
        vy, ly = _mode(g.ny, my, per)
        vz, lz = _mode(g.nz, mz, False)
        v = (vx[:, None, None] * vy[None, :, None] * vz[None, None, :]).ravel()
        mu = V * (1 + g.kh * lx / g.dx**2 + g.kh * ly / g.dy**2 + g.kv * lz / dzu**2)
        Av = A.matvec(v)
        assert np.linalg.norm(Av - mu * v) <= 1e-13 * mu * np.linalg.norm(v)
        # ... and the solver returns v / mu for b = v
        res = oracle.pcg(A, oracle.line_blocks(A, g.nz), v, rtol=1e-14)
        np.testing.assert_allclose(res["x"], v / mu, rtol=0, atol=1e-11 * np.abs(v / mu).max())


def _manufactured_error(N, K_v, q_coarse, N0):
    # u = sin(pi x) sin(pi y) sin(pi z) on the unit cube with Dirichlet u = 0;
    # -div(diag(1,1,K_v) grad u) + u = (1 + 2 pi^2 + K_v pi^2) u = f.
    # The right-hand side is the cell integral of f, the unknowns approximate
    # cell averages of u.  The vertical grading keeps one fixed mapping
    # z(xi) as the grid is refined (q_N = q_coarse^(N0/N)).
    q = q_coarse ** (N0 / N)
    g = oracle.Grid(N, N, N, 1.0 / N, 1.0 / N, 1.0, q, 1.0, K_v, False, False)
    dz = oracle.vertical_spacing(N, 1.0, q)
    zf = np.concatenate([[0.0], np.cumsum(dz)])
    xf = np.linspace(0, 1, N + 1)
    Ix = (np.cos(np.pi * xf[:-1]) - np.cos(np.pi * xf[1:])) / np.pi
    Iz = (np.cos(np.pi * zf[:-1]) - np.cos(np.pi * zf[1:])) / np.pi
    cell_int = (Ix[:, None, None] * Ix[None, :, None] * Iz[None, None, :]).ravel()
    vol = np.tile(g.dx * g.dy * dz, N * N)
    c = 1 + 2 * np.pi**2 + K_v * np.pi**2
    res = oracle.solve(g, c * cell_int, rtol=1e-13)
    avg = cell_int / vol
    return np.abs(res["x"] - avg).max() / np.abs(avg).max()


@pytest.mark.parametrize("K_v,q0", [(1.0, 1.3), (50.0, 1.5)])
def test_manufactured_solution_second_order(K_v, q0):
    e = [_manufactured_error(N, K_v, q0, 8) for N in (8, 16, 32)]
    rates = [np.log2(e[i] / e[i + 1]) for i in range(2)]
    assert e[2] < 5e-3
    assert min(rates) > 1.7, (e, rates)


def test_row_apply_matches_assembled_rows():
    rng = np.random.default_rng(11)
    for g in small_grids():
        A = oracle.assemble(g)
        x = rng.standard_normal(g.n)
        y = A.matvec(x).reshape(g.nx, g.ny, g.nz)
        for _ in range(10):
            i, j, k = rng.integers(g.nx), rng.integers(g.ny), rng.integers(g.nz)
            assert oracle.row_apply(g, i, j, k, x) == pytest.approx(y[i, j, k], rel=1e-14, abs=1e-14)


# ------------------------------------------------------ preconditioner ---

def test_single_column_preconditioner_is_the_operator():
    # with one horizontal cell there are no couplings to drop: M == A
    g = oracle.Grid(1, 1, 9, 0.5, 0.25, 1.0, 1.05, 1.0, 30.0, False, False)
    A = oracle.assemble(g)
    M = oracle.line_blocks(A, g.nz)
    Md = np.diag(M.di) + np.diag(M.lo[1:], -1) + np.diag(M.up[:-1], 1)
    assert np.array_equal(Md, dense(A))


@pytest.mark.parametrize("g", small_grids(), ids=lambda g: f"{g.nx}x{g.ny}x{g.nz}")
def test_line_blocks_keep_only_column_couplings(g):
    A = dense(oracle.assemble(g))
    M = oracle.line_blocks(oracle.assemble(g), g.nz)
    col = np.arange(g.n) // g.nz
    same = col[:, None] == col[None, :]
    Md = np.diag(M.di) + np.diag(M.lo[1:], -1) + np.diag(M.up[:-1], 1)
    np.testing.assert_array_equal(Md, np.where(same, A, 0.0))


@pytest.mark.parametrize("g", small_grids(), ids=lambda g: f"{g.nx}x{g.ny}x{g.nz}")
def test_thomas_matches_dense_lu(g):
    A = oracle.assemble(g)
    M = oracle.line_blocks(A, g.nz)
    Md = np.diag(M.di) + np.diag(M.lo[1:], -1) + np.diag(M.up[:-1], 1)
    r = np.random.default_rng(5).standard_normal(g.n)
    z = oracle.line_solve(M, r)
    zd = np.linalg.solve(Md, r)
    np.testing.assert_allclose(z, zd, rtol=1e-13, atol=1e-13 * np.abs(zd).max())


def test_single_level_line_preconditioner_is_jacobi():
    g = oracle.grid_from_ratio(5, 4, 1, 1e3, periodic=False)
    A = oracle.assemble(g)
    M = oracle.line_blocks(A, 1)
    r = np.random.default_rng(1).standard_normal(g.n)
    np.testing.assert_allclose(oracle.line_solve(M, r), r / np.diag(dense(A)), rtol=1e-15)


# ---------------------------------------------------------------- PCG ---

@pytest.mark.parametrize("g", small_grids(), ids=lambda g: f"{g.nx}x{g.ny}x{g.nz}")
def test_pcg_matches_dense_cholesky(g):
    A = oracle.assemble(g)
    b = si.rhs_uniform(g.nx, g.ny, g.nz, 0)
    res = oracle.pcg(A, oracle.line_blocks(A, g.nz), b, rtol=1e-14)
    assert res["status"] == "converged"
    xd = sla.cho_solve(sla.cho_factor(dense(A)), b)
    assert np.linalg.norm(res["x"] - xd) <= 1e-12 * np.linalg.norm(xd)


def test_no_horizontal_coupling_converges_in_one_iteration():
    # K_h = 0 makes A block diagonal, so M = A and z_0 = A^{-1} r_0 exactly
    g = oracle.Grid(6, 5, 16, 1 / 6, 1 / 5, 1.0, 1.05, 0.0, 1e3, False, False)
    A = oracle.assemble(g)
    res = oracle.pcg(A, oracle.line_blocks(A, g.nz), si.rhs_uniform(6, 5, 16, 3), rtol=1e-12)
    assert res["status"] == "converged" and res["iterations"] == 1


def test_zero_rhs_returns_zero_immediately():
    g = oracle.grid_from_ratio(4, 4, 4, 1e2)
    A = oracle.assemble(g)
    res = oracle.pcg(A, oracle.line_blocks(A, 4), np.zeros(g.n))
    assert res["iterations"] == 0 and res["status"] == "converged"
    assert not res["x"].any()


def test_max_iter_status():
    g = oracle.grid_from_ratio(8, 8, 8, 1e2)
    A = oracle.assemble(g)
    res = oracle.pcg(A, oracle.line_blocks(A, 8), si.rhs_uniform(8, 8, 8, 0), rtol=1e-14, max_iter=2)
    assert res["status"] == "max_iter" and res["iterations"] == 2


def test_true_residual_meets_tolerance():
    g = oracle.grid_from_ratio(16, 16, 16, 1e3)
    res = oracle.solve(g, si.rhs_uniform(16, 16, 16, 4), rtol=1e-8)
    assert res["rel_res"] < 1e-8
    assert res["rel_res_true"] < 1.01e-8


def test_cg_orthogonality_conjugacy_and_error_bound():
    g = oracle.grid_from_ratio(5, 6, 7, 1e1, q=1.05)
    A = oracle.assemble(g)
    M = oracle.line_blocks(A, g.nz)
    b = si.rhs_uniform(g.nx, g.ny, g.nz, 9)
    res = oracle.pcg(A, M, b, rtol=1e-10, trace=True)
    tr = res["trace"]
    k = res["iterations"]
    assert k >= 4
    X, R, Z, P = tr[:, 0], tr[:, 1], tr[:, 2], tr[:, 3]
    # residuals are M^{-1}-orthogonal: <r_i, z_j> = 0 (i != j)
    G = R @ Z.T
    nr = np.sqrt(np.abs(np.diag(G)))
    off = np.abs(G - np.diag(np.diag(G))) / np.outer(nr, nr)
    assert off.max() < 1e-8
    # search directions are A-conjugate
    AP = np.stack([A.matvec(p) for p in P[:-1]])
    C = P[:-1] @ AP.T
    nc = np.sqrt(np.diag(C))
    offc = np.abs(C - np.diag(np.diag(C))) / np.outer(nc, nc)
    assert offc.max() < 1e-8
    # A-norm error decreases monotonically and obeys the Chebyshev bound
    Ad = dense(A)
    xs = np.linalg.solve(Ad, b)
    err = np.array([np.sqrt((xs - x) @ Ad @ (xs - x)) for x in X])
    assert np.all(np.diff(err) < 0)
    Md = np.diag(M.di) + np.diag(M.lo[1:], -1) + np.diag(M.up[:-1], 1)
    ev = sla.eigh(Ad, Md, eigvals_only=True)
    kap = ev.max() / ev.min()
    rho = (np.sqrt(kap) - 1) / (np.sqrt(kap) + 1)
    for i, e in enumerate(err):
        assert e <= 2 * rho**i * err[0] * (1 + 1e-10)


def _interleaved_pcg(A, M, b, rtol, max_iter):
    """Alg. InterleavedPCG with the fused kernels of Algs. InterleavedApply and
    InterleavedPrec, written with whole-vector operations.  Readings: start
    with r = b - A u, p = q = 0, alpha = 0, kappa_old = 1; the forward
    substitution starts at level 0; on exit u still lacks alpha*p, which is
    added once."""
    u = np.zeros(A.n)
    r = b - A.matvec(u)
    p = np.zeros(A.n)
    q = np.zeros(A.n)
    alpha, kappa_old = 0.0, 1.0
    r0 = np.linalg.norm(r)
    xs = []
    for it in range(max_iter + 1):
        r = r - alpha * q
        z = oracle.line_solve(M, r)
        R, kappa = np.linalg.norm(r), r @ z
        xs.append(u + alpha * p)           # the iterate this state stands for
        if R / r0 < rtol or it == max_iter:
            return u + alpha * p, it, xs
        beta = kappa / kappa_old
        kappa_old = kappa
        u = u + alpha * p
        p = z + beta * p
        q = A.matvec(z) + beta * q
        sigma = p @ q
        alpha = kappa_old / sigma


@pytest.mark.parametrize("g", small_grids()[:3], ids=lambda g: f"{g.nx}x{g.ny}x{g.nz}")
def test_interleaved_pcg_equals_standard_pcg(g):
    A = oracle.assemble(g)
    M = oracle.line_blocks(A, g.nz)
    b = si.rhs_uniform(g.nx, g.ny, g.nz, 2)
    std = oracle.pcg(A, M, b, rtol=1e-12, trace=True)
    x, it, xs = _interleaved_pcg(A, M, b, 1e-12, 100)
    assert it == std["iterations"]
    for k, xk in enumerate(xs):
        ref = std["trace"][k, 0]
        assert np.linalg.norm(xk - ref) <= 1e-11 * max(np.linalg.norm(ref), 1e-300) + 1e-14
    assert np.linalg.norm(x - std["x"]) <= 1e-11 * np.linalg.norm(std["x"])


# ---------------------------------------------------------- generator ---

def test_generator_matches_published_splitmix64_vectors():
    with open(os.path.join(GOLDEN, "splitmix64.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    for row in rows:
        seed = int(row[0], 0)
        want = [int(v, 0) for v in row[1:]]
        got = [int(v) for v in si.splitmix64(seed, np.arange(len(want)))]
        assert got == want


def test_generator_ranges_and_independence_of_chunks():
    u = si.uniform_pm1(0, 1 << 16)
    assert u.min() >= -1 and u.max() < 1 and abs(u.mean()) < 0.02
    tail = si.uniform_pm1(0, 100, start=5000)
    np.testing.assert_array_equal(tail, u[5000:5100])


def test_torch_generator_equals_numpy_generator_on_cpu():
    torch = pytest.importorskip("torch")
    for seed, n, start in ((0, 5000, 0), (1234567, 3000, 10**6), (2**63 + 9, 100, 7)):
        a = si.uniform_pm1(seed, n, start)
        b = si.uniform_pm1_torch(seed, n, start, device="cpu").numpy()
        np.testing.assert_array_equal(a, b)


# ------------------------------------------------------ true residual ---
# orc_residual_norm is what every full-size GPU check leans on (the exit test
# of Alg. InterleavedPCG is on the 2-norm of r = b - A x), so it is pinned by
# facts that do not come from the oracle's own CSR loop.

@pytest.mark.parametrize("per", [False, True])
def test_residual_norm_closed_form_on_eigenvectors(per):
    # b = v (a closed-form eigenvector, A v = mu v) and x = c v give
    # ||b - A x|| = |1 - c mu| ||v|| exactly in exact arithmetic: this pins
    # the square root, the sign of A x and every term of the sum
    g = oracle.Grid(6, 5, 8, 0.3, 0.45, 2.0, 1.0, 1.7, 55.0, per, per)
    A = oracle.assemble(g)
    dzu = g.H / g.nz
    V = g.dx * g.dy * dzu
    for mx, my, mz in [(1, 1, 1), (2, 3, 5), (5, 4, 8)]:
        vx, lx = _mode(g.nx, mx, per)
        vy, ly = _mode(g.ny, my, per)
        vz, lz = _mode(g.nz, mz, False)
        v = (vx[:, None, None] * vy[None, :, None] * vz[None, None, :]).ravel()
        mu = V * (1 + g.kh * lx / g.dx**2 + g.kh * ly / g.dy**2 + g.kv * lz / dzu**2)
        nv = np.sqrt(np.sum(v * v))
        for c in (0.0, 0.25 / mu, 1.0 / mu, 3.0 / mu):
            expect = abs(1.0 - c * mu) * nv
            got = oracle.residual_norm(A, v, c * v)
            assert abs(got - expect) <= 1e-12 * nv, (c * mu, got, expect)


@pytest.mark.parametrize("g", small_grids(), ids=lambda g: f"{g.nx}x{g.ny}x{g.nz}")
def test_residual_norm_equals_dense_product_and_is_homogeneous(g):
    A = oracle.assemble(g)
    D = dense(A)
    rng = np.random.default_rng(17)
    for _ in range(3):
        b, x = rng.standard_normal(g.n), rng.standard_normal(g.n)
        ref = np.linalg.norm(b - D @ x)
        got = oracle.residual_norm(A, b, x)
        assert abs(got - ref) <= 1e-13 * ref
        # degree-one homogeneity (a sum of squares would scale by 4, a sum of
        # absolute values would not match the dense 2-norm above)
        assert abs(oracle.residual_norm(A, 2 * b, 2 * x) - 2 * got) <= 1e-13 * got
        # x = 0: the norm of b itself
        assert abs(oracle.residual_norm(A, b, np.zeros(g.n)) - np.linalg.norm(b)) <= \
            1e-14 * np.linalg.norm(b)
        # x = A^{-1} b from a dense solve: zero up to rounding
        xd = np.linalg.solve(D, b)
        assert oracle.residual_norm(A, b, xd) <= 1e-12 * np.linalg.norm(b)


def test_residual_norm_agrees_with_the_solvers_true_residual():
    # orc_pcg reports ||b - A x|| / ||r0|| of its own iterate, computed in
    # its own code; the stand-alone function must give the same number
    for g in small_grids():
        A = oracle.assemble(g)
        b = si.rhs_uniform(g.nx, g.ny, g.nz, 6)
        for k in (1, 2, 5):
            res = oracle.pcg(A, oracle.line_blocks(A, g.nz), b, rtol=0.0, max_iter=k)
            got = oracle.residual_norm(A, b, res["x"]) / res["r0"]
            assert abs(got - res["rel_res_true"]) <= 1e-12 * res["rel_res_true"] + 1e-300
