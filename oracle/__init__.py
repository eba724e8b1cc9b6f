"""CPU oracle for the line-preconditioned CG solver of arXiv 1302.7193.

TEST INFRASTRUCTURE ONLY: the test-suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only callers.  The product path
(the HIP library and its binding) never imports this package, and this
package imports nothing from the product.

The arithmetic lives in ``pcg_oracle.c`` (plain FP64 C, one file); this module
only marshals numpy arrays through ctypes.  What each function follows in the
paper:

* ``assemble``       Sec. 3.1, eqs. ModelEqnCubedSphere / DiagonalMatrix /
                     TridiagonalMatrix, written as an explicit finite-volume
                     CSR matrix on a flat graded grid (uniform or stretched
                     tensor-product horizontal cells).
* ``line_blocks``    Sec. 4.1: the preconditioner is A with the couplings
                     between vertical columns dropped.
* ``line_solve``     Sec. 4.2: one tridiagonal (Thomas) solve per column.
* ``pcg``            Sec. 4.1 standard preconditioned CG, exit test of
                     Alg. InterleavedPCG (||r||/||r0|| < rtol or ||r|| < atol).

Pins: see ``tests/test_oracle_pins.py`` (symmetry, definiteness, closed-form
eigenpairs, manufactured-solution convergence, dense direct solves, CG
invariants, the K_h = 0 and n_z = 1 special cases).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pcg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                               "-fno-fast-math", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    lib = ctypes.CDLL(build())
    lib.orc_vertical_spacing.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp]
    lib.orc_vertical_spacing.restype = None
    lib.orc_kv_from_ratio.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_int]
    lib.orc_kv_from_ratio.restype = ctypes.c_double
    geo = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
           ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
           ctypes.c_int, ctypes.c_int]
    lib.orc_assemble.argtypes = geo + [_i64p, _i32p, _dp]
    lib.orc_assemble.restype = ctypes.c_long
    lib.orc_csr_matvec.argtypes = [ctypes.c_long, _i64p, _i32p, _dp, _dp, _dp]
    lib.orc_csr_matvec.restype = None
    lib.orc_line_blocks.argtypes = [ctypes.c_long, ctypes.c_int, _i64p, _i32p, _dp, _dp, _dp, _dp]
    lib.orc_line_blocks.restype = None
    lib.orc_line_solve.argtypes = [ctypes.c_long, ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.orc_line_solve.restype = None
    lib.orc_pcg.argtypes = [ctypes.c_long, ctypes.c_int, _i64p, _i32p, _dp, _dp, _dp, _dp,
                            _dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp, _dp]
    lib.orc_pcg.restype = ctypes.c_int
    lib.orc_residual_norm.argtypes = [ctypes.c_long, _i64p, _i32p, _dp, _dp, _dp]
    lib.orc_residual_norm.restype = ctypes.c_double
    lib.orc_row_apply.argtypes = geo + [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp]
    lib.orc_row_apply.restype = ctypes.c_double
    geo_w = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_double,
             ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int]
    lib.orc_assemble_geom.argtypes = geo_w + [_i64p, _i32p, _dp]
    lib.orc_assemble_geom.restype = ctypes.c_long
    lib.orc_row_apply_geom.argtypes = geo_w + [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp]
    lib.orc_row_apply_geom.restype = ctypes.c_double
    _lib = lib
    return lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass(frozen=True)
class Grid:
    """Flat tensor-product grid: n_x*n_y horizontal cells of size dx*dy, n_z
    levels over height H graded with ratio q (finest at k = 0), diffusion
    K_h horizontally and K_v vertically, periodic or Dirichlet sides.
    Optional ``xw`` / ``yw`` (tuples of n_x / n_y widths) make the horizontal
    grid stretched; dx and dy are then unused."""
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    H: float
    q: float
    kh: float
    kv: float
    per_x: bool = False
    per_y: bool = False
    xw: tuple | None = None
    yw: tuple | None = None

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def stretched(self) -> bool:
        return self.xw is not None or self.yw is not None

    def widths(self):
        xw = np.full(self.nx, self.dx) if self.xw is None else _f64(self.xw)
        yw = np.full(self.ny, self.dy) if self.yw is None else _f64(self.yw)
        assert xw.shape == (self.nx,) and yw.shape == (self.ny,)
        return xw, yw

    def args(self):
        return (self.nx, self.ny, self.nz, self.dx, self.dy, self.H, self.q,
                self.kh, self.kv, int(self.per_x), int(self.per_y))

    def args_w(self, xw, yw):
        return (self.nx, self.ny, self.nz, _d(xw), _d(yw), self.H, self.q,
                self.kh, self.kv, int(self.per_x), int(self.per_y))


def kv_from_ratio(gamma2: float, kh: float, dx: float, H: float, nz: int) -> float:
    return _load().orc_kv_from_ratio(gamma2, kh, dx, H, nz)


def grid_from_ratio(nx, ny, nz, gamma2, q=1.05, periodic=False, H=1.0, kh=1.0) -> Grid:
    """Unit-square horizontal extent (dx = 1/n_x, dy = 1/n_y), K_v set from
    the anisotropy ratio gamma^2 at the mean vertical spacing."""
    dx, dy = 1.0 / nx, 1.0 / ny
    return Grid(nx, ny, nz, dx, dy, H, q, kh, kv_from_ratio(gamma2, kh, dx, H, nz),
                periodic, periodic)


def vertical_spacing(nz: int, H: float, q: float) -> np.ndarray:
    dz = np.empty(nz)
    _load().orc_vertical_spacing(nz, H, q, _d(dz))
    return dz


class CSR:
    def __init__(self, n, row_ptr, col, val):
        self.n, self.row_ptr, self.col, self.val = n, row_ptr, col, val

    def matvec(self, x):
        x = _f64(x)
        y = np.empty(self.n)
        _load().orc_csr_matvec(self.n, self.row_ptr.ctypes.data_as(_i64p),
                               self.col.ctypes.data_as(_i32p), _d(self.val), _d(x), _d(y))
        return y

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))

    def ptrs(self):
        return (self.row_ptr.ctypes.data_as(_i64p), self.col.ctypes.data_as(_i32p), _d(self.val))


def assemble(g: Grid) -> CSR:
    n = g.n
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(7 * n, dtype=np.int32)
    val = np.zeros(7 * n, dtype=np.float64)
    if g.stretched:
        xw, yw = g.widths()
        nnz = _load().orc_assemble_geom(*g.args_w(xw, yw), row_ptr.ctypes.data_as(_i64p),
                                        col.ctypes.data_as(_i32p), _d(val))
    else:
        nnz = _load().orc_assemble(*g.args(), row_ptr.ctypes.data_as(_i64p),
                                   col.ctypes.data_as(_i32p), _d(val))
    return CSR(n, row_ptr, col[:nnz].copy(), val[:nnz].copy())


class LineBlocks:
    def __init__(self, nz, lo, di, up):
        self.nz, self.lo, self.di, self.up = nz, lo, di, up


def line_blocks(A: CSR, nz: int) -> LineBlocks:
    lo, di, up = np.empty(A.n), np.empty(A.n), np.empty(A.n)
    _load().orc_line_blocks(A.n, nz, *A.ptrs(), _d(lo), _d(di), _d(up))
    return LineBlocks(nz, lo, di, up)


def line_solve(M: LineBlocks, r) -> np.ndarray:
    r = _f64(r)
    z = np.empty_like(r)
    work = np.empty(2 * M.nz)
    _load().orc_line_solve(r.size, M.nz, _d(M.lo), _d(M.di), _d(M.up), _d(r), _d(z), _d(work))
    return z


PCG_STATUS = {0: "converged", 1: "max_iter", 2: "breakdown"}


def pcg(A: CSR, M: LineBlocks, b, x0=None, rtol=1e-8, atol=0.0, max_iter=10000,
        trace=False) -> dict:
    """Standard PCG; returns dict(x, iterations, rel_res, r0, rel_res_true,
    status[, trace]) where trace has shape (iterations+1, 4, n) holding
    (x_k, r_k, z_k, p_k)."""
    b = _f64(b)
    x = np.zeros(A.n) if x0 is None else _f64(x0).copy()
    out = np.zeros(4)
    tr = np.zeros((max_iter + 1, 4, A.n)) if trace else None
    st = _load().orc_pcg(A.n, M.nz, *A.ptrs(), _d(M.lo), _d(M.di), _d(M.up), _d(b), _d(x),
                         rtol, atol, max_iter, _d(out),
                         _d(tr) if trace else ctypes.cast(None, _dp))
    res = dict(x=x, iterations=int(out[0]), rel_res=out[1], r0=out[2],
               rel_res_true=out[3], status=PCG_STATUS[st])
    if trace:
        res["trace"] = tr[: res["iterations"] + 1]
    return res


def residual_norm(A: CSR, b, x) -> float:
    return _load().orc_residual_norm(A.n, *A.ptrs(), _d(_f64(b)), _d(_f64(x)))


def row_apply(g: Grid, i: int, j: int, k: int, x) -> float:
    """(A x) at cell (i, j, k) without assembling A (for sampled checks on
    grids too large to assemble)."""
    if g.stretched:
        xw, yw = g.widths()
        return _load().orc_row_apply_geom(*g.args_w(xw, yw), i, j, k, _d(_f64(x)))
    return _load().orc_row_apply(*g.args(), i, j, k, _d(_f64(x)))


def solve(g: Grid, b, rtol=1e-8, atol=0.0, max_iter=10000, x0=None) -> dict:
    """Assemble, build the preconditioner and run PCG."""
    A = assemble(g)
    M = line_blocks(A, g.nz)
    res = pcg(A, M, b, x0=x0, rtol=rtol, atol=atol, max_iter=max_iter)
    res["A"] = A
    return res
