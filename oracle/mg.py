"""Tensor-product multigrid preconditioner for the oracle.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: the test-suite,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` are the
only callers; nothing here is shared with the HIP path.

The paper names this as the way forward (Sec. 1 and Sec. 8): a geometric
multigrid in the tensor-product spirit, where vertical line relaxation (the
preconditioner of Sec. 4.1) is the smoother and only the horizontal grid is
coarsened, the missing pieces being the intergrid operators.  It gives no
further detail, so every choice below is a reading, written out plainly:

* Levels: level 0 is the given grid; level l+1 merges 2 x 2 horizontal cells
  of level l (widths of neighbouring cells summed), keeping every vertical
  column, for as long as n_x and n_y are both even and both halves have at
  least ``MIN_CELLS`` cells.  At most ``max_levels`` levels (0: no limit).
* Coarse operators: the same finite-volume discretisation on the coarse
  grid (``oracle.assemble``), not a Galerkin product.
* Prolongation P: each fine column takes the values of its parent coarse
  column (piecewise constant in the horizontal; unknowns are cell values).
  Restriction: P transposed, i.e. a coarse residual is the sum of its four
  children's residuals (residuals are cell integrals).
* Smoother: damped vertical-line Jacobi, z <- z + omega M^{-1}(r - A z),
  omega = 0.8, with M the line preconditioner of the level.
* V-cycle on level l for residual r: one pre-smoothing sweep from z = 0,
  restriction of the residual, the V-cycle on level l+1, prolongation of its
  result added to z, one post-smoothing sweep.  On the coarsest level
  ``COARSE_SWEEPS`` sweeps from z = 0.  Pre- and post-smoothing match, so
  the V-cycle is a symmetric operator (pinned in the tests, with its
  definiteness).
* The Krylov loop is the same preconditioned CG (Sec. 4.1); the V-cycle
  replaces M^{-1}.
"""
from __future__ import annotations

import numpy as np

from . import CSR, Grid, assemble, line_blocks, line_solve

OMEGA = 0.8
MIN_CELLS = 4
COARSE_SWEEPS = 4


def coarse_grid(g: Grid) -> Grid | None:
    """The next coarser level of g, or None if g is the coarsest."""
    if g.nx % 2 or g.ny % 2 or g.nx // 2 < MIN_CELLS or g.ny // 2 < MIN_CELLS:
        return None
    xw, yw = g.widths()
    xc = xw[0::2] + xw[1::2]
    yc = yw[0::2] + yw[1::2]
    if g.stretched:
        return Grid(g.nx // 2, g.ny // 2, g.nz, 0.0, 0.0, g.H, g.q, g.kh, g.kv, g.per_x,
                    g.per_y, tuple(xc), tuple(yc))
    return Grid(g.nx // 2, g.ny // 2, g.nz, 2.0 * g.dx, 2.0 * g.dy, g.H, g.q, g.kh, g.kv,
                g.per_x, g.per_y)


def levels(g: Grid, max_levels: int = 0) -> list[Grid]:
    out = [g]
    while max_levels <= 0 or len(out) < max_levels:
        c = coarse_grid(out[-1])
        if c is None:
            break
        out.append(c)
    return out


def parent_index(gf: Grid, gc: Grid) -> np.ndarray:
    """For every fine cell (i, j, k), the index of coarse cell (i/2, j/2, k)."""
    idx = np.arange(gf.n)
    k = idx % gf.nz
    col = idx // gf.nz
    i, j = col // gf.ny, col % gf.ny
    return ((i // 2) * gc.ny + j // 2) * gc.nz + k


def prolong(gf: Grid, gc: Grid, zc) -> np.ndarray:
    return np.asarray(zc, dtype=np.float64)[parent_index(gf, gc)]


def restrict(gf: Grid, gc: Grid, r) -> np.ndarray:
    out = np.zeros(gc.n)
    np.add.at(out, parent_index(gf, gc), np.asarray(r, dtype=np.float64))
    return out


class Hierarchy:
    """Grids, operators and line preconditioners of every level."""

    def __init__(self, g: Grid, max_levels: int = 0, omega: float = OMEGA):
        self.grids = levels(g, max_levels)
        self.A = [assemble(x) for x in self.grids]
        self.M = [line_blocks(a, x.nz) for a, x in zip(self.A, self.grids)]
        self.omega = omega

    def smooth(self, l: int, r, z):
        """One damped line-Jacobi sweep z + omega M^{-1}(r - A z)."""
        return z + self.omega * line_solve(self.M[l], r - self.A[l].matvec(z))

    def vcycle(self, r, l: int = 0) -> np.ndarray:
        r = np.asarray(r, dtype=np.float64)
        z = self.omega * line_solve(self.M[l], r)          # pre-smoothing from zero
        if l == len(self.grids) - 1:
            for _ in range(COARSE_SWEEPS - 1):
                z = self.smooth(l, r, z)
            return z
        gf, gc = self.grids[l], self.grids[l + 1]
        rc = restrict(gf, gc, r - self.A[l].matvec(z))
        z = z + prolong(gf, gc, self.vcycle(rc, l + 1))
        return self.smooth(l, r, z)                          # post-smoothing


def pcg(A: CSR, prec, b, rtol=1e-8, atol=0.0, max_iter=10000) -> dict:
    """Standard preconditioned CG (Sec. 4.1) with any preconditioner
    callable; same exit test as ``oracle.pcg`` (||r||/||r0|| < rtol or
    ||r|| < atol on the recursively updated residual)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros(A.n)
    r = b.copy()
    r0 = np.linalg.norm(r)
    rn = r0
    it, status = 0, "max_iter"
    if r0 == 0.0 or r0 < atol:
        return dict(x=x, iterations=0, rel_res=0.0, r0=r0, status="converged")
    z = prec(r)
    p = z.copy()
    rho = r @ z
    while it < max_iter:
        q = A.matvec(p)
        pq = p @ q
        if not pq > 0:
            status = "breakdown"
            break
        alpha = rho / pq
        x += alpha * p
        r -= alpha * q
        it += 1
        rn = np.linalg.norm(r)
        if rn / r0 < rtol or rn < atol:
            status = "converged"
            break
        z = prec(r)
        rho_new = r @ z
        p = z + (rho_new / rho) * p
        rho = rho_new
    return dict(x=x, iterations=it, rel_res=rn / r0, r0=r0, status=status)


def solve(g: Grid, b, rtol=1e-8, max_iter=10000, max_levels: int = 0) -> dict:
    """PCG with the V-cycle preconditioner on grid g."""
    h = Hierarchy(g, max_levels)
    res = pcg(h.A[0], h.vcycle, b, rtol=rtol, max_iter=max_iter)
    res["levels"] = len(h.grids)
    res["A"] = h.A[0]
    return res
