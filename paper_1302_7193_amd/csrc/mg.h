// Tensor-product multigrid preconditioner (gfx950).
//
// Sec. 1 and Sec. 8 of the paper name the next step: a geometric multigrid
// in the tensor-product spirit, with the vertical line relaxation of
// Sec. 4.1 as the smoother and only the horizontal grid coarsened.  Level
// l+1 merges 2 x 2 horizontal cells of level l and keeps every vertical
// column, so every level is the same kind of operator (the column kernels'
// stencil and line solve apply unchanged with the level's geometry).
// Prolongation is piecewise constant in the horizontal (a fine column takes
// its parent's values), restriction its transpose (a coarse residual is the
// sum of its four children's), and the smoother is damped line Jacobi.
//
// The kernels and their dispatch; mg_f64.hip and mg_f32.hip instantiate
// them for one precision each (two translation units compile in parallel).
//
// Kernels, each over one level and fused to read every vector once:
//   k_mg_pre       t = omega M^{-1} r            (FUSED: r -= alpha q first,
//                                                 as kernel B of the fused
//                                                 iteration does)
//   k_mg_restrict  r_c = P^T (r - A t)           (one coarse column per lane
//                                                 segment: four children)
//   k_mg_post      w = t + P z_c;                (PROLONG: the correction is
//                  z = w + omega M^{-1}(r - A w)  added as neighbours load)
//                  FINAL: R = <r,r>, kappa = <r,z>; exit test; beta
// A sweep reads neighbouring columns of its input iterate, so it writes a
// different vector (t and z alternate).
// A V-cycle is pre / restrict down the levels, sweeps on the coarsest, and
// post back up; the fused iteration ends its kernel-B work with the fine
// level's FINAL post-smoothing.
#pragma once

#include "column.h"

namespace pcg {
namespace {

// NT: the vectors read or written once per sweep (r, q and the result) go
// with the nontemporal hint, the iterate whose neighbour columns are re-read
// and the coarse vectors without it.  W: one column per wavefront (L = 64,
// column index scalar), as in the fused kernels.

// Writes t = a.io2 from r (FUSED: from r or b with the update of kernel B,
// r written back to a.io1).
template <typename T, int M, bool V, bool G, bool FUSED, bool NT, bool W>
__global__ __launch_bounds__(kBlock) void k_mg_pre(ColArgs a)
{
    const Geom& g = a.g;
    const int L = W ? kWave : a.L;
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    int64_t rhs, blk;
    split_rhs(t, a.blocks_per_rhs, rhs, blk);
    SolverState* s = a.st ? a.st + rhs : nullptr;
    if (s && s->flag != kRunning) return;
    const int64_t off = rhs * g.n;
    const T* src;
    T* r = nullptr;
    const T* q = nullptr;
    T alpha = T(0);
    bool first = false, store_r = false;
    if constexpr (FUSED) {
        first = s->iter == 0;
        const bool from_b = first && s->zero_start;
        src = static_cast<const T*>(from_b ? a.in1 : a.io1) + off;
        r = static_cast<T*>(a.io1) + off;
        store_r = !(from_b && a.in1 == a.io1);
        q = static_cast<const T*>(a.io4) + off;
        alpha = T(s->alpha);
    } else {
        src = static_cast<const T*>(a.in0) + off;
    }
    T* z = static_cast<T*>(a.io2) + off;
    const T* lu = static_cast<const T*>(a.lu);
    const T omega = T(a.omega);
    const Lane p = lane_pos<M>(L);
    const SolveCoef<T, M, G> sc = load_solve<T, M, V, G>(g, a, p.k0);
    int64_t t0, t1;
    block_tiles(g, L, blk, a.blocks_per_rhs, t0, t1);
    for (int64_t tile = t0; tile < t1; ++tile) {
        const Col c = make_col<G>(g, W ? wave_col(tile, p) : tile_col(tile, p, L), a.hgeo);
        T rc[M], zc[M];
        ld<T, M, V, NT>(src, c.idx, c.ok, p.k0, g.nz, rc);
        if constexpr (FUSED) {
            if (!first) {
                T qc[M];
                ld<T, M, V, NT>(q, c.idx, c.ok, p.k0, g.nz, qc);
#pragma unroll
                for (int i = 0; i < M; ++i) rc[i] = rc[i] - alpha * qc[i];
            }
            if (!first || store_r) st<T, M, V, NT>(r, c.idx, c.ok, p.k0, g.nz, rc);
        }
        line_solve<T, M, V, G>(g, c, p.l, L, p.k0, lu, sc, rc, zc);
#pragma unroll
        for (int i = 0; i < M; ++i) zc[i] *= omega;
        st<T, M, V, NT>(z, c.idx, c.ok, p.k0, g.nz, zc);
    }
}

// Tiles of the coarse level a.g; the fine level is a.g2 (geometry a.hgeo2);
// reads r = a.in0 and t = a.in1 of the fine level, writes a.io0.
template <typename T, int M, bool V, bool G, bool NT, bool W>
__global__ __launch_bounds__(kBlock) void k_mg_restrict(ColArgs a)
{
    const Geom& gc = a.g;
    const Geom& gf = a.g2;
    const int L = W ? kWave : a.L;
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    int64_t rhs, blk;
    split_rhs(t, a.blocks_per_rhs, rhs, blk);
    if (a.st && a.st[rhs].flag != kRunning) return;
    const T* r = static_cast<const T*>(a.in0) + rhs * gf.n;
    const T* z = static_cast<const T*>(a.in1) + rhs * gf.n;
    T* rc_out = static_cast<T*>(a.io0) + rhs * gc.n;
    const Lane p = lane_pos<M>(L);
    const VertCoef<T, M> vc = load_vert<T, M, V>(gf, static_cast<const T*>(a.vert), p.k0);
    int64_t t0, t1;
    block_tiles(gc, L, blk, a.blocks_per_rhs, t0, t1);
    for (int64_t tile = t0; tile < t1; ++tile) {
        const Col cp = make_col<false>(gc, W ? wave_col(tile, p) : tile_col(tile, p, L));   // the coarse column
        T acc[M];
#pragma unroll
        for (int i = 0; i < M; ++i) acc[i] = T(0);
        if constexpr (M * sizeof(T) <= 16) {   // one 16-byte chunk per lane and vector
            // the 2x2 children (child = 2 di + dj) and their z: a child's
            // neighbours towards its siblings are those siblings (a coarse
            // level has at least 4 cells per direction), so besides them only
            // the eight outer neighbours are loaded: 12 columns of z, not 20
            Col c[4];
            T zf[4][M];
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) {
                c[ch] = make_col_ij<G>(gf, 2 * cp.i + (ch >> 1), 2 * cp.j + (ch & 1), cp.ok,
                                       a.hgeo2);
                ld<T, M, V>(z, c[ch].idx, c[ch].ok, p.k0, gf.nz, zf[ch]);
            }
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) {
                const int di = ch >> 1, dj = ch & 1;
                T az[M], rf[M];
                stencil_nb<T, M, G>(gf, c[ch], p.l, L, zf[ch], vc,
                                    [&](int dir, int64_t col, bool ok, T (&o)[M]) {
                                        // direction 0..3: i-1, i+1, j-1, j+1
                                        const int sib = dir == 0 ? (di == 1 ? ch - 2 : -1)
                                                      : dir == 1 ? (di == 0 ? ch + 2 : -1)
                                                      : dir == 2 ? (dj == 1 ? ch - 1 : -1)
                                                                 : (dj == 0 ? ch + 1 : -1);
                                        if (sib >= 0) {
#pragma unroll
                                            for (int i = 0; i < M; ++i) o[i] = zf[sib][i];
                                        } else {
                                            ld<T, M, V>(z, col, ok, p.k0, gf.nz, o);
                                        }
                                    },
                                    az);
                ld<T, M, V, NT>(r, c[ch].idx, c[ch].ok, p.k0, gf.nz, rf);
#pragma unroll
                for (int i = 0; i < M; ++i) acc[i] += rf[i] - az[i];
            }
        } else {
            // two children at a time, each loading its own neighbours (with
            // more levels per lane the shared form above holds too many
            // registers: all four children at once held 137 VGPRs)
#pragma unroll 2
            for (int ch = 0; ch < 4; ++ch) {
                const Col c = make_col_ij<G>(gf, 2 * cp.i + (ch >> 1), 2 * cp.j + (ch & 1),
                                             cp.ok, a.hgeo2);
                T zf[M], az[M], rf[M];
                ld<T, M, V>(z, c.idx, c.ok, p.k0, gf.nz, zf);
                stencil<T, M, V, G>(gf, c, p.l, L, p.k0, z, zf, vc, az);
                ld<T, M, V, NT>(r, c.idx, c.ok, p.k0, gf.nz, rf);
#pragma unroll
                for (int i = 0; i < M; ++i) acc[i] += rf[i] - az[i];
            }
        }
        st<T, M, V>(rc_out, cp.idx, cp.ok, p.k0, gc.nz, acc);
    }
}

// Coarse column (of level gc) containing fine column (i, j).
__device__ __forceinline__ int64_t parent_ij(const Geom& gc, int i, int j)
{
    return (int64_t)(i >> 1) * gc.ny + (j >> 1);
}

// Reads r = a.in0, the iterate t = a.io3 and (PROLONG) the coarse
// correction a.in1 on level a.g2; writes z = a.io2 (never t).
template <typename T, int M, bool V, bool G, bool PROLONG, bool FINAL, bool NT, bool W>
__global__ __launch_bounds__(kBlock) void k_mg_post(ColArgs a)
{
    const Geom& g = a.g;
    const Geom& gc = a.g2;
    const int L = W ? kWave : a.L;
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    int64_t rhs, blk;
    split_rhs(t, a.blocks_per_rhs, rhs, blk);
    SolverState* s = a.st ? a.st + rhs : nullptr;
    if (s && s->flag != kRunning) return;
    const int64_t off = rhs * g.n;
    const T* r = static_cast<const T*>(a.in0) + off;
    const T* zin = static_cast<const T*>(a.io3) + off;
    T* z = static_cast<T*>(a.io2) + off;
    const T* zc = PROLONG ? static_cast<const T*>(a.in1) + rhs * gc.n : nullptr;
    const T* lu = static_cast<const T*>(a.lu);
    const T omega = T(a.omega);
    const Lane p = lane_pos<M>(L);
    const VertCoef<T, M> vc = load_vert<T, M, V>(g, static_cast<const T*>(a.vert), p.k0);
    const SolveCoef<T, M, G> sc = load_solve<T, M, V, G>(g, a, p.k0);
    double acc[2] = {0.0, 0.0};
    int64_t t0, t1;
    block_tiles(g, L, blk, a.blocks_per_rhs, t0, t1);
    for (int64_t tile = t0; tile < t1; ++tile) {
        const Col c = make_col<G>(g, W ? wave_col(tile, p) : tile_col(tile, p, L), a.hgeo);
        // parents of the column and of its neighbours (periodic wrap as in
        // make_col; absent neighbours are never loaded)
        const int im = c.i > 0 ? c.i - 1 : g.nx - 1, ip = c.i < g.nx - 1 ? c.i + 1 : 0;
        const int jm = c.j > 0 ? c.j - 1 : g.ny - 1, jp = c.j < g.ny - 1 ? c.j + 1 : 0;
        // the corrected iterate t + P z_c on a column whose parent is pc
        auto load_z = [&](int64_t col, bool ok, int64_t pc, T (&o)[M]) {
            ld<T, M, V>(zin, col, ok, p.k0, g.nz, o);
            if constexpr (PROLONG) {
                T q[M];
                ld<T, M, V>(zc, pc, ok, p.k0, g.nz, q);
#pragma unroll
                for (int i = 0; i < M; ++i) o[i] += q[i];
            }
        };
        T zo[M], az[M], rc[M], dz[M];
        load_z(c.idx, c.ok, parent_ij(gc, c.i, c.j), zo);
        stencil_nb<T, M, G>(g, c, p.l, L, zo, vc,
                            [&](int dir, int64_t col, bool ok, T (&o)[M]) {
                                const int64_t pc = dir == 0   ? parent_ij(gc, im, c.j)
                                                   : dir == 1 ? parent_ij(gc, ip, c.j)
                                                   : dir == 2 ? parent_ij(gc, c.i, jm)
                                                              : parent_ij(gc, c.i, jp);
                                load_z(col, ok, pc, o);
                            },
                            az);
        ld<T, M, V, NT>(r, c.idx, c.ok, p.k0, g.nz, rc);
#pragma unroll
        for (int i = 0; i < M; ++i) az[i] = rc[i] - az[i];
        line_solve<T, M, V, G>(g, c, p.l, L, p.k0, lu, sc, az, dz);
#pragma unroll
        for (int i = 0; i < M; ++i) zo[i] += omega * dz[i];
        st<T, M, V, NT>(z, c.idx, c.ok, p.k0, g.nz, zo);
        if constexpr (FINAL) {
#pragma unroll
            for (int i = 0; i < M; ++i) {
                acc[0] += double(rc[i]) * double(rc[i]);
                acc[1] += double(rc[i]) * double(zo[i]);
            }
        }
    }
    if constexpr (FINAL) {
        double tot[2];
        if (publish<2>(acc, a.part + rhs * a.blocks_per_rhs * kRedSlots, blk, a.blocks_per_rhs,
                       &s->ticket, a.red_mode, tot)) {
            if (threadIdx.x == 0) finish_prec(s, tot[0], tot[1]);
        }
    }
}

template <typename T, int M, bool V, bool G, bool NT, bool W>
const void* mg_func_m(Kind kind)
{
    switch (kind) {
    case Kind::MgPre: return reinterpret_cast<const void*>(&k_mg_pre<T, M, V, G, false, NT, W>);
    case Kind::MgPreFused: return reinterpret_cast<const void*>(&k_mg_pre<T, M, V, G, true, NT, W>);
    case Kind::MgRestrict: return reinterpret_cast<const void*>(&k_mg_restrict<T, M, V, G, NT, W>);
    case Kind::MgPost:
        return reinterpret_cast<const void*>(&k_mg_post<T, M, V, G, true, false, NT, W>);
    case Kind::MgPostFinal:
        return reinterpret_cast<const void*>(&k_mg_post<T, M, V, G, true, true, NT, W>);
    case Kind::MgSmooth:
        return reinterpret_cast<const void*>(&k_mg_post<T, M, V, G, false, false, NT, W>);
    case Kind::MgSmoothFinal:
        return reinterpret_cast<const void*>(&k_mg_post<T, M, V, G, false, true, NT, W>);
    default: return nullptr;
    }
}

template <typename T, int M, bool V, bool G>
const void* mg_func_n(Kind kind, bool nt, bool w)
{
    // the nontemporal variants exist only where the hint is used: one
    // 16-byte chunk per lane and vector
    if constexpr (M * sizeof(T) == 16) {
        if (w) return nt ? mg_func_m<T, M, V, G, true, true>(kind) : mg_func_m<T, M, V, G, false, true>(kind);
        return nt ? mg_func_m<T, M, V, G, true, false>(kind) : mg_func_m<T, M, V, G, false, false>(kind);
    } else {
        return w ? mg_func_m<T, M, V, G, false, true>(kind) : mg_func_m<T, M, V, G, false, false>(kind);
    }
}

template <typename T, int M>
const void* mg_func_v(Kind kind, const ColArgs& a, bool nt)
{
    const bool vec = (a.g.nz % M == 0) && ((M * sizeof(T)) % 16 == 0) &&
                     ((a.g.nz * sizeof(T)) % 16 == 0);
    const bool w = a.L == kWave;
    if (a.hgeo || a.hgeo2)
        return vec ? mg_func_n<T, M, true, true>(kind, nt, w) : mg_func_n<T, M, false, true>(kind, nt, w);
    return vec ? mg_func_n<T, M, true, false>(kind, nt, w) : mg_func_n<T, M, false, false>(kind, nt, w);
}

}  // namespace

template <typename T>
const void* mg_func(Kind kind, const ColArgs& a, int64_t batch)
{
    const int M = a.L > 0 ? (a.g.nz + a.L - 1) / a.L : 0;
    int Mp = 1;
    while (Mp < M) Mp <<= 1;
    // the fine level's vectors of a large problem, as in the fused kernels
    // (restriction: the fine level is a.g2)
    const Geom& fine = kind == Kind::MgRestrict ? a.g2 : a.g;
    const bool nt = fine.n * batch * (int64_t)sizeof(T) >= kStreamBytes && Mp * sizeof(T) == 16;
    switch (Mp) {
    case 1: return mg_func_v<T, 1>(kind, a, nt);
    case 2: return mg_func_v<T, 2>(kind, a, nt);
    case 4: return mg_func_v<T, 4>(kind, a, nt);
    case 8: return mg_func_v<T, 8>(kind, a, nt);
    case 16: return mg_func_v<T, 16>(kind, a, nt);
    default: return nullptr;
    }
}

}  // namespace pcg
