"""Element- and column-wise comparison helpers for the GPU parity tests.

A norm over the whole vector dilutes an error confined to a few columns by
sqrt(columns hit / columns), so the checks below bound every element, or
every column, separately.
"""
import numpy as np

import oracle


def abs_product(M, z):
    """|M| |z| for the column blocks M of oracle.line_blocks."""
    az = np.abs(z)
    t = np.abs(M.di) * az
    t[1:] += np.abs(M.lo[1:]) * az[:-1]
    t[:-1] += np.abs(M.up[:-1]) * az[1:]
    return t


def line_solve_bound(M, z_ref, u, c):
    """Componentwise forward-error bound c u (M^{-1} |M| |z|)_i of a solve of
    M z = r with componentwise backward error c u |M| (first order).  The
    column blocks are M-matrices (positive diagonal, non-positive
    couplings, strictly diagonally dominant), so M^{-1} >= 0 and the bound
    is one more line solve; it holds for perturbed coefficients (FP32
    tables) and for any order of evaluation that is backward stable."""
    return c * u * oracle.line_solve(M, abs_product(M, z_ref))


def column_backward_errors(M, z, r, nz):
    """Per column: ||M_c z_c - r_c||_inf / (||M_c||_inf ||z_c||_inf)."""
    res = M.di * z
    res[1:] += M.lo[1:] * z[:-1]
    res[:-1] += M.up[:-1] * z[1:]
    res = np.abs(res - r).reshape(-1, nz).max(axis=1)
    normM = (np.abs(M.di) + np.abs(M.lo) + np.abs(M.up)).reshape(-1, nz).max(axis=1)
    normz = np.abs(z).reshape(-1, nz).max(axis=1)
    return res / (normM * normz + 1e-300)


def column_rel_errors(z, want, nz):
    """Per column: ||z_c - w_c|| / max(||w_c||, rms column norm of w)."""
    e = np.linalg.norm((z - want).reshape(-1, nz), axis=1)
    w = np.linalg.norm(want.reshape(-1, nz), axis=1)
    rms = np.sqrt(np.mean(w * w))
    return e / np.maximum(w, rms + 1e-300)
