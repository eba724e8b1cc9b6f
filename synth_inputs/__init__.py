"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

This module holds input data recipes only; it contains none of the solver's
arithmetic.  Every value is a pure function of (seed, logical index), so any
subset can be regenerated independently.

Generator: SplitMix64 (S. Vigna, public-domain reference implementation,
https://prng.di.unimi.it/splitmix64.c).  Element ``idx`` of the stream with
seed ``s`` is the output of the generator whose state starts at ``s`` after
``idx + 1`` steps, i.e. ``mix(s + (idx + 1) * 0x9E3779B97F4A7C15)`` with

    z ^= z >> 30;  z *= 0xBF58476D1CE4E5B9;
    z ^= z >> 27;  z *= 0x94D049BB133111EB;
    z ^= z >> 31.

A float in [0, 1) is the top 53 bits times 2^-53; U[-1, 1) is 2u - 1.

Logical index of cell (i, j, k) on an n_x x n_y x n_z grid is
``(i * n_y + j) * n_z + k`` (vertical columns stored contiguously).
"""
from __future__ import annotations

import math

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)
_CHUNK = 1 << 22


def splitmix64(seed: int, idx: np.ndarray) -> np.ndarray:
    """Raw 64-bit outputs for stream ``seed`` at positions ``idx``."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (idx + np.uint64(1)) * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, start: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.float64)
    for s in range(0, count, _CHUNK):
        e = min(count, s + _CHUNK)
        z = splitmix64(seed, np.arange(start + s, start + e, dtype=np.uint64))
        out[s:e] = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return out


def uniform_pm1(seed: int, count: int, start: int = 0) -> np.ndarray:
    """i.i.d. U[-1, 1) values for logical indices start .. start+count-1."""
    u = uniform01(seed, start, count)
    u *= 2.0
    u -= 1.0
    return u


def rhs_uniform(nx: int, ny: int, nz: int, seed: int) -> np.ndarray:
    """Right-hand side b with i.i.d. U[-1, 1) entries (one per cell)."""
    return uniform_pm1(seed, nx * ny * nz)


def rhs_smooth_noise(nx: int, ny: int, nz: int, seed: int, noise: float = 0.01) -> np.ndarray:
    """Smooth sinusoidal field plus uniform noise:
    b = sin(pi*(i+1/2)/n_x) * sin(pi*(j+1/2)/n_y) * sin(pi*(k+1/2)/n_z)
        + noise * U[-1, 1),
    with the sine taken over the logical (index) coordinates of the cell."""
    sx = np.sin(np.pi * (np.arange(nx) + 0.5) / nx)
    sy = np.sin(np.pi * (np.arange(ny) + 0.5) / ny)
    sz = np.sin(np.pi * (np.arange(nz) + 0.5) / nz)
    n = nx * ny * nz
    out = np.empty(n, dtype=np.float64)
    col = nz
    rows_per_chunk = max(1, _CHUNK // (ny * nz))
    for i0 in range(0, nx, rows_per_chunk):
        i1 = min(nx, i0 + rows_per_chunk)
        smooth = (sx[i0:i1, None, None] * sy[None, :, None] * sz[None, None, :]).ravel()
        start = i0 * ny * col
        out[start:start + smooth.size] = smooth + noise * uniform_pm1(seed, smooth.size, start)
    return out


# ---- the same streams generated on a torch device (large workloads) ----
# int64 arithmetic wraps modulo 2^64 on the device; logical right shifts are
# an arithmetic shift followed by a mask.  Element-for-element equal to the
# numpy functions above (tested).

def _i64(v: int) -> int:
    v &= 0xFFFFFFFFFFFFFFFF
    return v - (1 << 64) if v >= (1 << 63) else v


def _srl(z, k: int):
    import torch
    return torch.bitwise_and(torch.bitwise_right_shift(z, k), (1 << (64 - k)) - 1)


def uniform_pm1_torch(seed: int, count: int, start: int = 0, device="cuda", out=None):
    """U[-1, 1) values for logical indices start .. start+count-1 as a float64
    tensor on `device` (optionally written into `out`)."""
    import torch
    if out is None:
        out = torch.empty(count, dtype=torch.float64, device=device)
    g, m1, m2 = _i64(int(GOLDEN)), _i64(int(M1)), _i64(int(M2))
    sd = _i64(seed)
    chunk = 1 << 24
    for s in range(0, count, chunk):
        e = min(count, s + chunk)
        z = torch.arange(start + s + 1, start + e + 1, dtype=torch.int64, device=out.device)
        z.mul_(g).add_(sd)
        z = torch.bitwise_xor(z, _srl(z, 30)).mul_(m1)
        z = torch.bitwise_xor(z, _srl(z, 27)).mul_(m2)
        z = torch.bitwise_xor(z, _srl(z, 31))
        u = _srl(z, 11).to(torch.float64)
        out[s:e] = u.mul_(2.0 / 9007199254740992.0).sub_(1.0)
    return out


def rhs_uniform_torch(nx, ny, nz, seed, device="cuda", out=None):
    return uniform_pm1_torch(seed, nx * ny * nz, 0, device, out)


def rhs_smooth_noise_torch(nx, ny, nz, seed, noise=0.01, device="cuda"):
    import torch
    out = uniform_pm1_torch(seed, nx * ny * nz, 0, device)
    out.mul_(noise)
    ar = lambda m: torch.sin(torch.pi * (torch.arange(m, dtype=torch.float64, device=out.device) + 0.5) / m)
    sx, sy, sz = ar(nx), ar(ny), ar(nz)
    o3 = out.view(nx, ny, nz)
    for i in range(nx):
        o3[i].add_(sx[i] * sy[:, None] * sz[None, :])
    return out


def widths_sine(n: int, amp: float = 0.5, length: float = 1.0) -> np.ndarray:
    """Smoothly stretched horizontal cell widths: w_i proportional to
    1 + amp*sin(2*pi*(i + 1/2)/n), scaled so they sum to ``length``.  The
    ratio of the largest to the smallest width is about (1+amp)/(1-amp), and
    the variation is periodic, so the same widths suit periodic sides."""
    w = 1.0 + amp * np.sin(2.0 * np.pi * (np.arange(n) + 0.5) / n)
    return w * (length / w.sum())


def widths_graded(n: int, ratio: float = 1.05, length: float = 1.0) -> np.ndarray:
    """Cell widths refined towards both ends (walls): w_i proportional to
    ratio**min(i, n-1-i), scaled to sum to ``length``."""
    i = np.arange(n)
    w = ratio ** np.minimum(i, n - 1 - i).astype(np.float64)
    return w * (length / w.sum())


def widths_random(n: int, seed: int, lo: float = 0.5, hi: float = 1.5,
                  length: float = 1.0) -> np.ndarray:
    """Independent widths drawn uniformly from [lo, hi) (stream ``seed``),
    scaled to sum to ``length``; neighbouring cells differ arbitrarily."""
    w = lo + (hi - lo) * uniform01(seed, 0, n)
    return w * (length / w.sum())


def rhs_batch(nx: int, ny: int, nz: int, seeds) -> np.ndarray:
    """Stack of U[-1, 1) right-hand sides, one row per seed."""
    return np.stack([rhs_uniform(nx, ny, nz, s) for s in seeds])


def serving_trace(n_requests: int = 512, rate: float = 200.0, seed: int = 5,
                  sizes=(64, 128, 256, 512), levels=(32, 64, 128),
                  log_ratio=(2.0, 5.0), rhs_seed_base: int = 1000):
    """Synthetic request trace: Poisson arrivals with the given mean rate,
    horizontal size n x n drawn uniformly from ``sizes``, levels from
    ``levels``, anisotropy ratio log-uniform in 10**log_ratio, and the RHS
    seed ``rhs_seed_base + request id``.  All draws come from stream
    ``seed`` at fixed positions (4 per request)."""
    u = uniform01(seed, 0, 4 * n_requests).reshape(n_requests, 4)
    gaps = -np.log1p(-u[:, 0]) / rate
    arrivals = np.cumsum(gaps) - gaps[0]
    reqs = []
    for r in range(n_requests):
        nh = sizes[min(len(sizes) - 1, int(u[r, 1] * len(sizes)))]
        nzr = levels[min(len(levels) - 1, int(u[r, 2] * len(levels)))]
        g2 = 10.0 ** (log_ratio[0] + (log_ratio[1] - log_ratio[0]) * u[r, 3])
        reqs.append(dict(id=r, arrival=float(arrivals[r]), nx=nh, ny=nh, nz=nzr,
                         gamma2=float(g2), seed=rhs_seed_base + r))
    return reqs


def describe_trace(reqs) -> dict:
    n = np.array([q["nx"] * q["ny"] * q["nz"] for q in reqs], dtype=np.float64)
    return dict(requests=len(reqs), mean_unknowns=float(n.mean()),
                span_s=float(reqs[-1]["arrival"] - reqs[0]["arrival"]) if reqs else 0.0,
                log10_total=math.log10(float(n.sum())) if reqs else 0.0)
