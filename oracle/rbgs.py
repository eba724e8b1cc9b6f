"""Symmetric block Gauss-Seidel preconditioner for the oracle.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: the test-suite,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` are the
only callers; nothing here is shared with the HIP path.

Sec. 4.1 of the paper notes that block-SOR preconditioners can replace the
block-diagonal (vertical line) one, needing the inversion of the same
block-diagonal matrix plus one more sparse matrix-vector product.  Readings
taken here (the paper gives no details):

* the blocks are the vertical columns (the blocks of the line
  preconditioner), ordered red-black by horizontal position: column (i, j)
  is red when i + j is even;
* relaxation factor 1 (block Gauss-Seidel) and one forward plus one
  backward sweep, so the preconditioner is symmetric:
  M = (D + L) D^{-1} (D + U) with D the column blocks and L, U the
  couplings between columns of different colours in red-black order;
* every neighbour of a column must have the other colour, so a periodic
  direction needs an even number of cells.

Applied to r from zero: the red columns solve with r alone, the black
columns with r minus the couplings to the red result, and the red columns
again with r minus the couplings to the black result (the backward sweep's
black step would repeat the forward one and is left out).
"""
from __future__ import annotations

import numpy as np

from . import CSR, Grid, assemble, line_blocks, line_solve


def supported(g: Grid) -> bool:
    return not ((g.per_x and g.nx % 2) or (g.per_y and g.ny % 2))


def red_mask(g: Grid) -> np.ndarray:
    """True for the cells of red columns (i + j even)."""
    idx = np.arange(g.n)
    col = idx // g.nz
    i, j = col // g.ny, col % g.ny
    return (i + j) % 2 == 0


class RBGS:
    def __init__(self, g: Grid, A: CSR | None = None):
        if not supported(g):
            raise ValueError("red-black ordering needs an even size in periodic directions")
        self.g = g
        self.A = A if A is not None else assemble(g)
        self.M = line_blocks(self.A, g.nz)
        self.red = red_mask(g)

    def apply(self, r) -> np.ndarray:
        r = np.asarray(r, dtype=np.float64)
        red, black = self.red, ~self.red
        z_red = line_solve(self.M, np.where(red, r, 0.0)) * red
        rb = r - self.A.matvec(z_red)
        z_black = line_solve(self.M, np.where(black, rb, 0.0)) * black
        rr = r - self.A.matvec(z_black)
        z_red = line_solve(self.M, np.where(red, rr, 0.0)) * red
        return z_red + z_black
