// Column kernels of the line-preconditioned CG solver (gfx950): the operator,
// the line preconditioner, the start-up, the two fused kernels of
// Alg. InterleavedPCG, the exit correction, the refinement kernels of the
// mixed-precision form, their finalize launches, and the host-side
// dispatch.  The building blocks (work decomposition, stencil, line solve)
// are in column.h.  kernels_f64.hip and kernels_f32.hip instantiate the
// launchers for one precision each (two translation units that compile in
// parallel).
#pragma once

#include <algorithm>

#include "column.h"

namespace pcg {
namespace {

// Tiles a wavefront takes at a time in the kernels with a single input
// stream (the operator and the preconditioner alone, the first launches of
// kernels A and B): their loads are issued together before any arithmetic.
constexpr int kStepApply = 4, kStepPrecond = 4, kStepFirstA = 4, kStepFirstB = 4;
constexpr int kStepResidual = 4;   // the FP64 refinement residual (a stencil too)

inline int step_of(Kind k)
{
    switch (k) {
    case Kind::Apply: return kStepApply;
    case Kind::Precond: return kStepPrecond;
    case Kind::FusedApplyFirst: return kStepFirstA;
    case Kind::FusedPrecFirst: return kStepFirstB;
    case Kind::Residual64: return kStepResidual;
    default: return 1;
    }
}

// ---------------------------------------------------------------- kernels --

// Column c of wavefront step `tile` (U tiles per step): the column index of
// tile + u, or one past the grid (make_col then marks it absent) beyond t1.
// JS (one column per wavefront): the wavefront takes U consecutive columns
// of the step's 4U instead, so with n_y a multiple of U they lie in one row
// of the grid and share their inner y-neighbours (load_group).
template <bool W, int U, bool JS>
__device__ __forceinline__ int64_t step_col(const Geom& g, int64_t tile, int u, int64_t t1,
                                            const Lane& p, int L)
{
    if constexpr (JS) {
        const int c = __builtin_amdgcn_readfirstlane(
            (int)(tile * (kBlock / kWave) + p.wave * U + u));
        return c < t1 * (kBlock / kWave) ? int64_t(c) : g.nh;
    }
    const int64_t tu = tile + u;
    if (tu >= t1) return g.nh;
    return W ? wave_col(tu, p) : tile_col(tu, p, L);
}

// The geometry of a wavefront step's U columns.  JS: consecutive columns of
// one grid row (n_y a multiple of U, the step's first column a multiple of
// U), so one division by n_y places all of them.
template <bool G, bool W, int U, bool JS>
__device__ __forceinline__ void step_cols(const Geom& g, int64_t tile, int64_t t1, const Lane& p,
                                          int L, const double* hgeo, Col (&c)[U])
{
    static_assert(!JS || (kBlock / kWave) % U == 0, "a step's first column must be a multiple of U");
    if constexpr (JS) {
        const int64_t c0 = step_col<W, U, true>(g, tile, 0, t1, p, L);
        const int64_t lim = t1 * (kBlock / kWave) < g.nh ? t1 * (kBlock / kWave) : g.nh;
        const uint32_t cc = c0 < lim ? uint32_t(c0) : 0u;
        const uint32_t i = cc / uint32_t(g.ny);
        const int j0 = int(cc - i * uint32_t(g.ny));
#pragma unroll
        for (int u = 0; u < U; ++u) c[u] = make_col_ij<G>(g, int(i), j0 + u, c0 + u < lim, hgeo);
    } else {
#pragma unroll
        for (int u = 0; u < U; ++u)
            c[u] = make_col<G>(g, step_col<W, U, false>(g, tile, u, t1, p, L), hgeo);
    }
}

// The stencil inputs of a wavefront step's U columns.  JS: the columns are
// consecutive in one row (see step_col), so column u's y-neighbours are
// columns u - 1 and u + 1 of the group, already loaded, and only the
// group's outer two are read; the loads are all issued before any use.
template <typename T, int M, bool V, int U, bool JS>
__device__ __forceinline__ void load_group(const Geom& g, const Col (&c)[U], int k0,
                                           const T* __restrict__ x, StencilIn<T, M> (&in)[U])
{
    if constexpr (!JS) {
#pragma unroll
        for (int u = 0; u < U; ++u) load_stencil<T, M, V>(g, c[u], k0, x, in[u]);
    } else {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            ld<T, M, V>(x, c[u].idx, c[u].ok, k0, g.nz, in[u].xc);
            ld<T, M, V>(x, c[u].im, c[u].ok && c[u].im >= 0, k0, g.nz, in[u].nb[0]);
            ld<T, M, V>(x, c[u].ip, c[u].ok && c[u].ip >= 0, k0, g.nz, in[u].nb[1]);
        }
        ld<T, M, V>(x, c[0].jm, c[0].ok && c[0].jm >= 0, k0, g.nz, in[0].nb[2]);
        ld<T, M, V>(x, c[U - 1].jp, c[U - 1].ok && c[U - 1].jp >= 0, k0, g.nz, in[U - 1].nb[3]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int t = 0; t < M; ++t) {
                if (u > 0) in[u].nb[2][t] = in[u - 1].xc[t];
                if (u < U - 1) in[u].nb[3][t] = in[u + 1].xc[t];
            }
        }
    }
}

// W: one column per wavefront (L = 64, column index scalar); NT: the
// vectors streamed once carry the nontemporal hint (x is not one of them:
// its columns are re-read as the horizontal neighbours of others).  U: each
// wavefront takes U tiles at a time and issues the loads of all of them
// before computing any: a kernel with one input stream otherwise keeps too
// few bytes in flight to cover the memory latency.
template <typename T, int M, bool V, bool G, bool NT, bool W, int U, bool JS>
__global__ __launch_bounds__(kBlock) void k_apply(ColArgs a)
{
    const Geom& g = a.g;
    const int L = W ? kWave : a.L;
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    int64_t rhs, blk;
    split_rhs(t, a.blocks_per_rhs, rhs, blk);
    if (a.st && a.st[rhs].flag != kRunning) return;   // inside a solve: stop when done
    const T* x = static_cast<const T*>(a.in0) + rhs * g.n;
    T* y = static_cast<T*>(a.io0) + rhs * g.n;
    const T* vert = static_cast<const T*>(a.vert);
    const Lane p = lane_pos<M>(L);
    const VertCoef<T, M> vc = load_vert<T, M, V>(g, vert, p.k0);
    int64_t t0, t1;
    block_tiles(g, L, blk, a.blocks_per_rhs, t0, t1);
    for (int64_t tile = t0; tile < t1; tile += U) {
        Col c[U];
        StencilIn<T, M> in[U];
        T yc[U][M];
        step_cols<G, W, U, JS>(g, tile, t1, p, L, a.hgeo, c);
        load_group<T, M, V, U, JS>(g, c, p.k0, x, in);
#pragma unroll
        for (int u = 0; u < U; ++u) stencil_in<T, M, G>(g, c[u], p.l, L, in[u], vc, yc[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) st<T, M, V, NT>(y, c[u].idx, c[u].ok, p.k0, g.nz, yc[u]);
    }
}

template <typename T, int M, bool V, bool G, bool NT, bool W, int U>
__global__ __launch_bounds__(kBlock) void k_precond(ColArgs a)
{
    const Geom& g = a.g;
    const int L = W ? kWave : a.L;
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    int64_t rhs, blk;
    split_rhs(t, a.blocks_per_rhs, rhs, blk);
    if (a.st && a.st[rhs].flag != kRunning) return;
    const T* r = static_cast<const T*>(a.in0) + rhs * g.n;
    T* z = static_cast<T*>(a.io0) + rhs * g.n;
    const T* lu = static_cast<const T*>(a.lu);
    const Lane p = lane_pos<M>(L);
    const SolveCoef<T, M, G> sc = load_solve<T, M, V, G>(g, a, p.k0);
    int64_t t0, t1;
    block_tiles(g, L, blk, a.blocks_per_rhs, t0, t1);
    for (int64_t tile = t0; tile < t1; tile += U) {
        Col c[U];
        T rc[U][M], zc[U][M];
        step_cols<G, W, U, false>(g, tile, t1, p, L, a.hgeo, c);
#pragma unroll
        for (int u = 0; u < U; ++u) ld<T, M, V, NT>(r, c[u].idx, c[u].ok, p.k0, g.nz, rc[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) line_solve<T, M, V, G>(g, c[u], p.l, L, p.k0, lu, sc, rc[u], zc[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) st<T, M, V, NT>(z, c[u].idx, c[u].ok, p.k0, g.nz, zc[u]);
    }
}

// r = b - A x; ZERO: x = 0, r = b (nothing to copy when b is r), p = q = 0.
template <typename T, int M, bool V, bool ZERO, bool G, bool NT, bool W>
__global__ __launch_bounds__(kBlock) void k_init(ColArgs a)
{
    const Geom& g = a.g;
    const int L = W ? kWave : a.L;
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    int64_t rhs, blk;
    split_rhs(t, a.blocks_per_rhs, rhs, blk);
    const int64_t off = rhs * g.n;
    T* x = static_cast<T*>(a.io0) + off;
    const T* b = static_cast<const T*>(a.in1) + off;
    T* r = static_cast<T*>(a.io1) + off;
    T* pp = static_cast<T*>(a.io3) + off;
    T* q = static_cast<T*>(a.io4) + off;
    const T* vert = static_cast<const T*>(a.vert);
    const bool in_place = a.in1 == a.io1;   // b already stored in r
    const Lane p = lane_pos<M>(L);
    const VertCoef<T, M> vc = load_vert<T, M, V>(g, vert, p.k0);
    int64_t t0, t1;
    block_tiles(g, L, blk, a.blocks_per_rhs, t0, t1);
    T zero[M];
#pragma unroll
    for (int i = 0; i < M; ++i) zero[i] = T(0);
    for (int64_t tile = t0; tile < t1; ++tile) {
        const Col c = make_col<G>(g, W ? wave_col(tile, p) : tile_col(tile, p, L), a.hgeo);
        if (ZERO) {
            st<T, M, V, NT>(x, c.idx, c.ok, p.k0, g.nz, zero);
            if (!in_place) {
                T bc[M];
                ld<T, M, V, NT>(b, c.idx, c.ok, p.k0, g.nz, bc);
                st<T, M, V, NT>(r, c.idx, c.ok, p.k0, g.nz, bc);
            }
        } else {
            T bc[M], rc[M], ax[M];
            StencilIn<T, M> in;
            ld<T, M, V, NT>(b, c.idx, c.ok, p.k0, g.nz, bc);
            load_stencil<T, M, V>(g, c, p.k0, x, in);
            stencil_in<T, M, G>(g, c, p.l, L, in, vc, ax);
#pragma unroll
            for (int i = 0; i < M; ++i) rc[i] = bc[i] - ax[i];
            st<T, M, V, NT>(r, c.idx, c.ok, p.k0, g.nz, rc);
        }
        if (ZERO) {   // the unfused iteration reads p and q; the fused one does not
            st<T, M, V, NT>(pp, c.idx, c.ok, p.k0, g.nz, zero);
            st<T, M, V, NT>(q, c.idx, c.ok, p.k0, g.nz, zero);
        }
    }
}

// Kernel B (Alg. InterleavedPrec): r -= alpha q; z = M^{-1} r;
// R = <r,r>, kappa = <r,z> (FP64 accumulation); scalar step: exit test, beta.
// FIRST (no iteration done yet): alpha = 0 and q is unset, so q is not read;
// with a zero start r is taken from b (no start-up kernel).  The first launch
// leaves r unchanged and does not store it: r is already in io1 (a start-up
// kernel wrote it, or b is r itself), or, with the line preconditioner
// (ColArgs::zswap), the second launch reads b again.
// W: one column per wavefront (L = 64, column index scalar).
template <typename T, int M, bool V, bool FIRST, bool G, bool NT, bool W, bool CZ = false>
__device__ __forceinline__ void fused_prec_body(const ColArgs& a, SolverState* s, int64_t rhs,
                                                int64_t blk, double (&acc)[2])
{
    const Geom& g = a.g;
    const int L = W ? kWave : a.L;
    const int64_t off = rhs * g.n;
    const bool from_b = s->zero_start && (FIRST || (a.zswap && s->iter == 1));
    const T* src = static_cast<const T*>(from_b ? a.in1 : a.io1) + off;
    T* r = static_cast<T*>(a.io1) + off;
    const bool store_r = !FIRST || (from_b && a.in1 != a.io1 && !a.zswap);
    T* z = static_cast<T*>((a.zswap && !FIRST) ? a.io3 : a.io2) + off;
    const T* q = static_cast<const T*>(a.io4) + off;
    const T* lu = static_cast<const T*>(a.lu);
    const T alpha = T(s->alpha);
    const Lane p = lane_pos<M>(L);
    const SolveCoef<T, M, G> sc = load_solve<T, M, V, G>(g, a, p.k0);
    int64_t t0, t1;
    block_tiles(g, L, blk, a.blocks_per_rhs, t0, t1);
    for (int64_t tile = t0; tile < t1; ++tile) {
        const Col c = make_col<G>(g, W ? wave_col(tile, p) : tile_col(tile, p, L), a.hgeo);
        T rc[M], zc[M];
        ld<T, M, V, NT>(src, c.idx, c.ok, p.k0, g.nz, rc);
        if (!FIRST) {
            T qc[M];
            ld<T, M, V, NT>(q, c.idx, c.ok, p.k0, g.nz, qc);
#pragma unroll
            for (int i = 0; i < M; ++i) rc[i] = rc[i] - alpha * qc[i];
        }
#pragma unroll
        for (int i = 0; i < M; ++i) acc[0] += double(rc[i]) * double(rc[i]);
        if (store_r) st<T, M, V, NT>(r, c.idx, c.ok, p.k0, g.nz, rc);
        line_solve<T, M, V, G>(g, c, p.l, L, p.k0, lu, sc, rc, zc);
#pragma unroll
        for (int i = 0; i < M; ++i) acc[1] += double(rc[i]) * double(zc[i]);
        // CZ: z without the nontemporal hint (ColArgs::cache_z): kernel A
        // reads it next
        st<T, M, V, NT && !CZ>(z, c.idx, c.ok, p.k0, g.nz, zc);
    }
}

template <typename T, int M, bool V, bool G, bool NT, bool W, bool CZ = false>
__device__ __forceinline__ void fused_prec_dev(const ColArgs& a, int64_t t)
{
    int64_t rhs, blk;
    split_rhs(t, a.blocks_per_rhs, rhs, blk);
    SolverState* s = a.st + rhs;
    if (s->flag != kRunning) return;
    double acc[2] = {0.0, 0.0};
    if (s->iter == 0) fused_prec_body<T, M, V, true, G, NT, W, CZ>(a, s, rhs, blk, acc);
    else fused_prec_body<T, M, V, false, G, NT, W, CZ>(a, s, rhs, blk, acc);
    double tot[2];
    if (publish<2>(acc, a.part + rhs * a.blocks_per_rhs * kRedSlots, blk, a.blocks_per_rhs,
                   &s->ticket, a.red_mode, tot)) {
        if (threadIdx.x == 0) finish_prec(s, tot[0], tot[1]);
    }
}

template <typename T, int M, bool V, bool G, bool NT, bool W, bool CZ>
__global__ __launch_bounds__(kBlock) void k_fused_prec(ColArgs a)
{
    fused_prec_dev<T, M, V, G, NT, W, CZ>(a, xcd_remap(blockIdx.x, gridDim.x));
}

// Kernel A (Alg. InterleavedApply): u += alpha p; p = z + beta p;
// q = A z + beta q; sigma = <p,q> (FP64); scalar step: alpha.
// FIRST: alpha = 0 and p = q = 0, so p = z, q = A z, and u keeps x0 (for a
// zero start u stays unwritten until the next launch sets u = alpha p); u, p
// and q are not read, and with zswap p = z is not stored (ColArgs::zswap).
template <typename T, int M, bool V, bool FIRST, bool G, bool NT, bool W>
__device__ __forceinline__ void fused_apply_body(const ColArgs& a, SolverState* s, int64_t rhs,
                                                 int64_t blk, double (&acc)[1])
{
    const Geom& g = a.g;
    const int L = W ? kWave : a.L;
    const int64_t off = rhs * g.n;
    T* u = static_cast<T*>(a.io0) + off;
    // z and p trade places after the first launch when zswap is set
    const bool swapped = a.zswap && !FIRST;
    const T* z = static_cast<const T*>(swapped ? a.io3 : a.io2) + off;
    T* pp = static_cast<T*>(swapped ? a.io2 : a.io3) + off;
    T* q = static_cast<T*>(a.io4) + off;
    const T* vert = static_cast<const T*>(a.vert);
    const T alpha = T(s->alpha), beta = T(s->beta);
    // zero start: u is not written by the first launch (it would be zero)
    // and the second sets u = alpha p instead of reading it
    const bool u_unset = s->zero_start && s->iter == 1;
    const Lane p = lane_pos<M>(L);
    const VertCoef<T, M> vc = load_vert<T, M, V>(g, vert, p.k0);
    int64_t t0, t1;
    block_tiles(g, L, blk, a.blocks_per_rhs, t0, t1);
    for (int64_t tile = t0; tile < t1; ++tile) {
        const Col c = make_col<G>(g, W ? wave_col(tile, p) : tile_col(tile, p, L), a.hgeo);
        T zc[M], az[M], pc[M], qc[M];
        ld<T, M, V>(z, c.idx, c.ok, p.k0, g.nz, zc);
        stencil<T, M, V, G>(g, c, p.l, L, p.k0, z, zc, vc, az);
        if (FIRST) {
#pragma unroll
            for (int i = 0; i < M; ++i) {
                pc[i] = zc[i];
                qc[i] = az[i];
                acc[0] += double(pc[i]) * double(qc[i]);
            }
        } else {
            T uc[M];
            if (u_unset) {
#pragma unroll
                for (int i = 0; i < M; ++i) uc[i] = T(0);
            } else {
                ld<T, M, V, NT>(u, c.idx, c.ok, p.k0, g.nz, uc);
            }
            ld<T, M, V, NT>(pp, c.idx, c.ok, p.k0, g.nz, pc);
            ld<T, M, V, NT>(q, c.idx, c.ok, p.k0, g.nz, qc);
#pragma unroll
            for (int i = 0; i < M; ++i) {
                uc[i] = uc[i] + alpha * pc[i];
                pc[i] = zc[i] + beta * pc[i];
                qc[i] = az[i] + beta * qc[i];
                acc[0] += double(pc[i]) * double(qc[i]);
            }
            st<T, M, V, NT>(u, c.idx, c.ok, p.k0, g.nz, uc);
        }
        if (!(FIRST && a.zswap)) st<T, M, V, NT>(pp, c.idx, c.ok, p.k0, g.nz, pc);
        st<T, M, V, NT>(q, c.idx, c.ok, p.k0, g.nz, qc);
    }
}

template <typename T, int M, bool V, bool G, bool NT, bool W>
__device__ __forceinline__ void fused_apply_dev(const ColArgs& a, int64_t t)
{
    int64_t rhs, blk;
    split_rhs(t, a.blocks_per_rhs, rhs, blk);
    SolverState* s = a.st + rhs;
    if (s->flag != kRunning) return;
    double acc[1] = {0.0};
    if (s->iter == 0) fused_apply_body<T, M, V, true, G, NT, W>(a, s, rhs, blk, acc);
    else fused_apply_body<T, M, V, false, G, NT, W>(a, s, rhs, blk, acc);
    double tot[1];
    if (publish<1>(acc, a.part + rhs * a.blocks_per_rhs * kRedSlots, blk, a.blocks_per_rhs,
                   &s->ticket, a.red_mode, tot)) {
        if (threadIdx.x == 0) finish_apply(s, tot[0]);
    }
}

template <typename T, int M, bool V, bool G, bool NT, bool W>
__global__ __launch_bounds__(kBlock) void k_fused_apply(ColArgs a)
{
    fused_apply_dev<T, M, V, G, NT, W>(a, xcd_remap(blockIdx.x, gridDim.x));
}

// First launch of kernel B in a solve (iteration 0: alpha = 0, q unset),
// compiled apart from the general kernel so that its wavefronts can take U
// tiles at a time (its loads issued together, the line solves of the U
// columns interleaved) without the general kernel's registers: r (or b on a
// zero start, ColArgs::x0_zero) in, z out, R = <r,r>, kappa = <r,z>, scalar
// step.  r is not stored (see fused_prec_body).  It runs once per solve, so
// its loads need not wait for the solver flag: the flag (set only for a
// right-hand side of a batch that is already done) is read alongside them
// and checked before anything is stored.
template <typename T, int M, bool V, bool G, bool NT, bool W, int U, bool CZ>
__global__ __launch_bounds__(kBlock) void k_fused_prec_first(ColArgs a)
{
    const Geom& g = a.g;
    const int L = W ? kWave : a.L;
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    int64_t rhs, blk;
    split_rhs(t, a.blocks_per_rhs, rhs, blk);
    SolverState* s = a.st + rhs;
    const int32_t flag = s->flag;
    const int64_t off = rhs * g.n;
    const T* src = static_cast<const T*>(a.x0_zero ? a.in1 : a.io1) + off;
    T* r = static_cast<T*>(a.io1) + off;
    const bool store_r = a.x0_zero && a.in1 != a.io1 && !a.zswap;
    T* z = static_cast<T*>(a.io2) + off;
    const T* lu = static_cast<const T*>(a.lu);
    const Lane p = lane_pos<M>(L);
    const SolveCoef<T, M, G> sc = load_solve<T, M, V, G>(g, a, p.k0);
    int64_t t0, t1;
    block_tiles(g, L, blk, a.blocks_per_rhs, t0, t1);
    double acc[2] = {0.0, 0.0};
    for (int64_t tile = t0; tile < t1; tile += U) {
        Col c[U];
        T rc[U][M], zc[U][M];
        step_cols<G, W, U, false>(g, tile, t1, p, L, a.hgeo, c);
#pragma unroll
        for (int u = 0; u < U; ++u) ld<T, M, V, NT>(src, c[u].idx, c[u].ok, p.k0, g.nz, rc[u]);
        if (flag != kRunning) return;   // the same in every thread of the workgroup
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int i = 0; i < M; ++i) acc[0] += double(rc[u][i]) * double(rc[u][i]);
            if (store_r) st<T, M, V, NT>(r, c[u].idx, c[u].ok, p.k0, g.nz, rc[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) line_solve<T, M, V, G>(g, c[u], p.l, L, p.k0, lu, sc, rc[u], zc[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int i = 0; i < M; ++i) acc[1] += double(rc[u][i]) * double(zc[u][i]);
            st<T, M, V, NT && !CZ>(z, c[u].idx, c[u].ok, p.k0, g.nz, zc[u]);   // CZ: fused_prec_body
        }
    }
    if (flag != kRunning) return;
    double tot[2];
    if (publish<2>(acc, a.part + rhs * a.blocks_per_rhs * kRedSlots, blk, a.blocks_per_rhs,
                   &s->ticket, a.red_mode, tot)) {
        if (threadIdx.x == 0) finish_prec(s, tot[0], tot[1]);
    }
}

// First launch of kernel A in a solve (iteration 0: alpha = 0, p = q = 0):
// p = z, q = A z, sigma = <z, A z>, scalar step; U tiles per wavefront
// step and the solver flag checked before the stores, as in
// k_fused_prec_first.  z stays in io2 and serves as p when ColArgs::zswap
// is set; otherwise p = z is stored.  u keeps x0 (a zero start leaves it
// unwritten until the next launch sets u = alpha p).
template <typename T, int M, bool V, bool G, bool NT, bool W, int U, bool JS>
__global__ __launch_bounds__(kBlock) void k_fused_apply_first(ColArgs a)
{
    const Geom& g = a.g;
    const int L = W ? kWave : a.L;
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    int64_t rhs, blk;
    split_rhs(t, a.blocks_per_rhs, rhs, blk);
    SolverState* s = a.st + rhs;
    const int32_t flag = s->flag;
    const int64_t off = rhs * g.n;
    const T* z = static_cast<const T*>(a.io2) + off;
    T* pp = static_cast<T*>(a.io3) + off;
    T* q = static_cast<T*>(a.io4) + off;
    const T* vert = static_cast<const T*>(a.vert);
    const Lane p = lane_pos<M>(L);
    const VertCoef<T, M> vc = load_vert<T, M, V>(g, vert, p.k0);
    int64_t t0, t1;
    block_tiles(g, L, blk, a.blocks_per_rhs, t0, t1);
    double acc[1] = {0.0};
    for (int64_t tile = t0; tile < t1; tile += U) {
        Col c[U];
        StencilIn<T, M> in[U];
        T az[U][M];
        step_cols<G, W, U, JS>(g, tile, t1, p, L, a.hgeo, c);
        load_group<T, M, V, U, JS>(g, c, p.k0, z, in);
#pragma unroll
        for (int u = 0; u < U; ++u) stencil_in<T, M, G>(g, c[u], p.l, L, in[u], vc, az[u]);
        if (flag != kRunning) return;   // the same in every thread of the workgroup
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int i = 0; i < M; ++i) acc[0] += double(in[u].xc[i]) * double(az[u][i]);
            if (!a.zswap) st<T, M, V, NT>(pp, c[u].idx, c[u].ok, p.k0, g.nz, in[u].xc);
            st<T, M, V, NT>(q, c[u].idx, c[u].ok, p.k0, g.nz, az[u]);
        }
    }
    if (flag != kRunning) return;
    double tot[1];
    if (publish<1>(acc, a.part + rhs * a.blocks_per_rhs * kRedSlots, blk, a.blocks_per_rhs,
                   &s->ticket, a.red_mode, tot)) {
        if (threadIdx.x == 0) finish_apply(s, tot[0]);
    }
}

// Exit correction u += alpha p (the fused iteration leaves u one step
// behind r).  Runs once: the last workgroup (or the finalize launch) marks
// it done.
template <typename T, int M, bool V, bool NT, bool W>
__device__ __forceinline__ void fixup_dev(const ColArgs& a, int64_t t)
{
    const Geom& g = a.g;
    const int L = W ? kWave : a.L;
    int64_t rhs, blk;
    split_rhs(t, a.blocks_per_rhs, rhs, blk);
    SolverState* s = a.st + rhs;
    // stopped before the first iteration: x = x0 (zero for a zero start, which
    // nothing has written yet -- also after a breakdown in the first kernel)
    const bool none = s->iter == 0;
    const bool stopped = s->flag == kConverged || s->flag == kMaxIter ||
                         (s->flag == kBreakdown && none);
    if (!stopped || s->fixed) return;
    if (none && !s->zero_start) return;
    // zero start stopped after one iteration: kernel A has not written u yet
    const bool u_unset = s->zero_start && s->iter == 1;
    const int64_t off = rhs * g.n;
    T* u = static_cast<T*>(a.io0) + off;
    const T* pp = static_cast<const T*>(a.zswap ? a.io2 : a.io3) + off;
    const T alpha = T(s->alpha);
    const Lane p = lane_pos<M>(L);
    int64_t t0, t1;
    block_tiles(g, L, blk, a.blocks_per_rhs, t0, t1);
    for (int64_t tile = t0; tile < t1; ++tile) {
        const Col c = make_col(g, W ? wave_col(tile, p) : tile_col(tile, p, L));
        T uc[M];
        if (none) {
#pragma unroll
            for (int i = 0; i < M; ++i) uc[i] = T(0);
        } else {
            T pc[M];
            if (u_unset) {
#pragma unroll
                for (int i = 0; i < M; ++i) uc[i] = T(0);
            } else {
                ld<T, M, V, NT>(u, c.idx, c.ok, p.k0, g.nz, uc);
            }
            ld<T, M, V, NT>(pp, c.idx, c.ok, p.k0, g.nz, pc);
#pragma unroll
            for (int i = 0; i < M; ++i) uc[i] += alpha * pc[i];
        }
        st<T, M, V, NT>(u, c.idx, c.ok, p.k0, g.nz, uc);
    }
    if (a.red_mode == 0) {   // mode 1: the finalize launch marks it done
        double acc[1] = {0.0}, tot[1];
        if (publish<1>(acc, a.part + rhs * a.blocks_per_rhs * kRedSlots, blk, a.blocks_per_rhs,
                       &s->ticket, 0, tot)) {
            if (threadIdx.x == 0) s->fixed = 1;
        }
    }
}

template <typename T, int M, bool V, bool NT, bool W>
__global__ __launch_bounds__(kBlock) void k_fixup(ColArgs a)
{
    fixup_dev<T, M, V, NT, W>(a, xcd_remap(blockIdx.x, gridDim.x));
}

// FP64 true residual: ||b - A x|| into state.aux (T = double only).
template <int M, bool V, bool G, bool NT, bool W>
__global__ __launch_bounds__(kBlock) void k_true_residual(ColArgs a)
{
    const Geom& g = a.g;
    const int L = W ? kWave : a.L;
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    int64_t rhs, blk;
    split_rhs(t, a.blocks_per_rhs, rhs, blk);
    SolverState* s = a.st + rhs;
    const double* x = static_cast<const double*>(a.in0) + rhs * g.n;
    const double* b = static_cast<const double*>(a.in1) + rhs * g.n;
    const double* vert = static_cast<const double*>(a.vert);
    const Lane p = lane_pos<M>(L);
    const VertCoef<double, M> vc = load_vert<double, M, V>(g, vert, p.k0);
    int64_t t0, t1;
    block_tiles(g, L, blk, a.blocks_per_rhs, t0, t1);
    double acc[1] = {0.0};
    for (int64_t tile = t0; tile < t1; ++tile) {
        const Col c = make_col<G>(g, W ? wave_col(tile, p) : tile_col(tile, p, L), a.hgeo);
        double ax[M], bc[M];
        StencilIn<double, M> in;
        ld<double, M, V, NT>(b, c.idx, c.ok, p.k0, g.nz, bc);
        load_stencil<double, M, V>(g, c, p.k0, x, in);
        stencil_in<double, M, G>(g, c, p.l, L, in, vc, ax);
#pragma unroll
        for (int i = 0; i < M; ++i) {
            const double d = bc[i] - ax[i];
            acc[0] += d * d;
        }
    }
    double tot[1];
    if (publish<1>(acc, a.part + rhs * a.blocks_per_rhs * kRedSlots, blk, a.blocks_per_rhs,
                       &s->ticket, a.red_mode, tot)) {
        if (threadIdx.x == 0) s->aux = sqrt(tot[0]);
    }
}

// Refinement residual: r64 = b - A x in FP64 (r64 = b when ZERO: x = 0 is
// not read), ||r64|| into state.rnorm (state.r0norm on the first call), FP32
// copy r32 = r64 * scale.  The FP32 vectors take the FP64 launch shape:
// chunks of M floats, aligned to their size whenever the FP64 ones are.
template <int M, bool V, bool ZERO, bool G, bool NT, bool W, int U, bool JS>
__device__ __forceinline__ void residual64_body(const ColArgs& a, SolverState* s, int64_t rhs,
                                                int64_t blk, double (&acc)[1])
{
    const Geom& g = a.g;
    const int L = W ? kWave : a.L;
    const double* x = static_cast<const double*>(a.in0) + rhs * g.n;
    const double* b = static_cast<const double*>(a.in1) + rhs * g.n;
    float* r32 = static_cast<float*>(a.out32) + rhs * g.n;
    const double* vert = static_cast<const double*>(a.vert);
    const double scale = s->aux;
    const Lane p = lane_pos<M>(L);
    const VertCoef<double, M> vc = load_vert<double, M, V>(g, vert, p.k0);
    int64_t t0, t1;
    block_tiles(g, L, blk, a.blocks_per_rhs, t0, t1);
    // U tiles per wavefront step, their loads issued together (see k_apply)
    for (int64_t tile = t0; tile < t1; tile += U) {
        Col c[U];
        double ax[U][M], bc[U][M];
        step_cols<G, W, U, JS>(g, tile, t1, p, L, a.hgeo, c);
#pragma unroll
        for (int u = 0; u < U; ++u) ld<double, M, V, NT>(b, c[u].idx, c[u].ok, p.k0, g.nz, bc[u]);
        if constexpr (ZERO) {
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int i = 0; i < M; ++i) ax[u][i] = 0.0;
        } else {
            StencilIn<double, M> in[U];
            load_group<double, M, V, U, JS>(g, c, p.k0, x, in);
#pragma unroll
            for (int u = 0; u < U; ++u) stencil_in<double, M, G>(g, c[u], p.l, L, in[u], vc, ax[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            float rc[M];
#pragma unroll
            for (int i = 0; i < M; ++i) {
                const double d = bc[u][i] - ax[u][i];
                acc[0] += d * d;
                rc[i] = float(d * scale);
            }
            st<float, M, V, NT>(r32, c[u].idx, c[u].ok, p.k0, g.nz, rc);
        }
    }
}

template <int M, bool V, bool G, bool NT, bool W, int U = 1, bool JS = false>
__device__ __forceinline__ void residual64_dev(const ColArgs& a, int64_t t)
{
    int64_t rhs, blk;
    split_rhs(t, a.blocks_per_rhs, rhs, blk);
    SolverState* s = a.st + rhs;
    if (s->flag != kRunning) return;
    double acc[1] = {0.0};
    if (a.x0_zero) residual64_body<M, V, true, G, NT, W, U, JS>(a, s, rhs, blk, acc);
    else residual64_body<M, V, false, G, NT, W, U, JS>(a, s, rhs, blk, acc);
    double tot[1];
    if (publish<1>(acc, a.part + rhs * a.blocks_per_rhs * kRedSlots, blk, a.blocks_per_rhs,
                       &s->ticket, a.red_mode, tot)) {
        if (threadIdx.x == 0) {
            const double rn = sqrt(tot[0]);
            s->rnorm = rn;
            if (s->iter == 0) s->r0norm = rn;
        }
    }
}

template <int M, bool V, bool G, bool NT, bool W, int U, bool JS>
__global__ __launch_bounds__(kBlock) void k_residual64(ColArgs a)
{
    residual64_dev<M, V, G, NT, W, U, JS>(a, xcd_remap(blockIdx.x, gridDim.x));
}

// Refinement update: x64 += (u32 + alpha p32) / scale, u32 being the inner
// solution without its pending exit correction alpha p (the inner solve runs
// no exit-correction kernel: the update folds it in, saving a pass over the
// FP32 vectors).  From the inner solve's state (zero start): u is valid
// after two or more iterations (unwritten before); alpha p is added when it
// stopped by the exit test or the iteration limit after at least one
// iteration (a breakdown leaves u as it is, like the exit correction).
// Both vectors are always read and the unused values selected away, so no
// branch separates the loads.  ZERO: x = 0 is not read.
template <int M, bool V, bool ZERO, bool NT, bool W>
__device__ __forceinline__ void update64_body(const ColArgs& a, const SolverState* s,
                                              const SolverState* si, int64_t rhs, int64_t blk)
{
    const Geom& g = a.g;
    const int L = W ? kWave : a.L;
    double* x = static_cast<double*>(a.io0) + rhs * g.n;
    const float* u32 = static_cast<const float*>(a.out32) + rhs * g.n;
    const float* p32 = static_cast<const float*>(a.in0) + rhs * g.n;
    const double inv_scale = 1.0 / s->aux;
    const bool u_valid = si->iter >= 2;
    const bool add_p = (si->flag == kConverged || si->flag == kMaxIter) && si->iter >= 1;
    const float alpha = add_p ? float(si->alpha) : 0.0f;
    const Lane p = lane_pos<M>(L);
    int64_t t0, t1;
    block_tiles(g, L, blk, a.blocks_per_rhs, t0, t1);
    for (int64_t tile = t0; tile < t1; ++tile) {
        const Col c = make_col(g, W ? wave_col(tile, p) : tile_col(tile, p, L));
        double xc[M];
        float uc[M], pc[M];
        if constexpr (ZERO) {
#pragma unroll
            for (int i = 0; i < M; ++i) xc[i] = 0.0;
        } else {
            ld<double, M, V, NT>(x, c.idx, c.ok, p.k0, g.nz, xc);
        }
        ld<float, M, V, NT>(u32, c.idx, c.ok, p.k0, g.nz, uc);
        ld<float, M, V, NT>(p32, c.idx, c.ok, p.k0, g.nz, pc);
#pragma unroll
        for (int i = 0; i < M; ++i) {
            const float ui = u_valid ? uc[i] : 0.0f;
            const float pi = add_p ? pc[i] : 0.0f;
            xc[i] += inv_scale * double(ui + alpha * pi);
        }
        keep_here(xc);
        st<double, M, V, NT>(x, c.idx, c.ok, p.k0, g.nz, xc);
    }
}

template <int M, bool V, bool NT, bool W>
__device__ __forceinline__ void update64_dev(const ColArgs& a, int64_t t)
{
    int64_t rhs, blk;
    split_rhs(t, a.blocks_per_rhs, rhs, blk);
    SolverState* s = a.st + rhs;
    if (s->flag != kRunning) return;
    const SolverState* si = a.st_in + rhs;
    if (a.x0_zero) update64_body<M, V, true, NT, W>(a, s, si, rhs, blk);
    else update64_body<M, V, false, NT, W>(a, s, si, rhs, blk);
}

template <int M, bool V, bool NT, bool W>
__global__ __launch_bounds__(kBlock) void k_update64(ColArgs a)
{
    update64_dev<M, V, NT, W>(a, xcd_remap(blockIdx.x, gridDim.x));
}

// Mode-1 reductions: one workgroup per right-hand side totals the published
// partial sums in the same order as mode 0 and performs the scalar step.
template <Kind K>
__device__ __forceinline__ void finalize_dev(const ColArgs& a, int64_t rhs)
{
    SolverState* s = a.st + rhs;
    const double* part = a.part + rhs * a.blocks_per_rhs * kRedSlots;
    if (K == Kind::Fixup) {
        if (threadIdx.x == 0 && (s->flag == kConverged || s->flag == kMaxIter ||
                                 (s->flag == kBreakdown && s->iter == 0)))
            s->fixed = 1;
        return;
    }
    if (K != Kind::TrueResidual && s->flag != kRunning) return;   // main kernel skipped
    if (K == Kind::FusedPrec) {
        double tot[2];
        sum_partials<2, false, kFinalThreads>(part, a.blocks_per_rhs, tot);
        if (threadIdx.x == 0) finish_prec(s, tot[0], tot[1]);
    } else {
        double tot[1];
        sum_partials<1, false, kFinalThreads>(part, a.blocks_per_rhs, tot);
        if (threadIdx.x == 0) {
            if (K == Kind::FusedApply) finish_apply(s, tot[0]);
            else if (K == Kind::TrueResidual) s->aux = sqrt(tot[0]);
            else if (K == Kind::Residual64) {
                s->rnorm = sqrt(tot[0]);
                if (s->iter == 0) s->r0norm = s->rnorm;
            }
        }
    }
}

template <Kind K>
__global__ __launch_bounds__(kFinalThreads) void k_finalize(ColArgs a)
{
    finalize_dev<K>(a, blockIdx.x);
}

inline bool has_finalize(Kind k)
{
    return k == Kind::FusedPrec || k == Kind::FusedApply || k == Kind::FusedPrecFirst ||
           k == Kind::FusedApplyFirst || k == Kind::Fixup ||
           k == Kind::TrueResidual || k == Kind::Residual64 || k == Kind::MgPostFinal ||
           k == Kind::MgSmoothFinal || k == Kind::RbRedFinal;
}

inline const void* finalize_func(Kind kind)
{
    switch (kind) {
    case Kind::FusedPrec:
    case Kind::FusedPrecFirst:
    case Kind::MgPostFinal:
    case Kind::MgSmoothFinal:
    case Kind::RbRedFinal: return reinterpret_cast<const void*>(&k_finalize<Kind::FusedPrec>);
    case Kind::FusedApply:
    case Kind::FusedApplyFirst: return reinterpret_cast<const void*>(&k_finalize<Kind::FusedApply>);
    case Kind::Fixup: return reinterpret_cast<const void*>(&k_finalize<Kind::Fixup>);
    case Kind::TrueResidual: return reinterpret_cast<const void*>(&k_finalize<Kind::TrueResidual>);
    case Kind::Residual64: return reinterpret_cast<const void*>(&k_finalize<Kind::Residual64>);
    default: return nullptr;
    }
}

template <typename T, int M, bool V, bool G, bool NT, bool W>
const void* main_func_m(Kind kind, bool js, bool cz)
{
    // columns sharing y-neighbours: one column per wavefront and n_y a
    // multiple of the step (the caller's js)
    constexpr bool kJs = W;
    switch (kind) {
    case Kind::Apply:
        if (kJs && js) return reinterpret_cast<const void*>(&k_apply<T, M, V, G, NT, W, kStepApply, kJs>);
        return reinterpret_cast<const void*>(&k_apply<T, M, V, G, NT, W, kStepApply, false>);
    case Kind::Precond:
        return reinterpret_cast<const void*>(&k_precond<T, M, V, G, NT, W, kStepPrecond>);
    case Kind::FusedPrecFirst:
        if (NT && cz)
            return reinterpret_cast<const void*>(&k_fused_prec_first<T, M, V, G, NT, W, kStepFirstB, true>);
        return reinterpret_cast<const void*>(&k_fused_prec_first<T, M, V, G, NT, W, kStepFirstB, false>);
    case Kind::FusedApplyFirst:
        if (kJs && js)
            return reinterpret_cast<const void*>(&k_fused_apply_first<T, M, V, G, NT, W, kStepFirstA, kJs>);
        return reinterpret_cast<const void*>(&k_fused_apply_first<T, M, V, G, NT, W, kStepFirstA, false>);
    case Kind::InitFull: return reinterpret_cast<const void*>(&k_init<T, M, V, false, G, NT, W>);
    case Kind::InitZero: return reinterpret_cast<const void*>(&k_init<T, M, V, true, false, NT, W>);
    case Kind::FusedPrec:
        if (NT && cz) return reinterpret_cast<const void*>(&k_fused_prec<T, M, V, G, NT, W, true>);
        return reinterpret_cast<const void*>(&k_fused_prec<T, M, V, G, NT, W, false>);
    case Kind::FusedApply: return reinterpret_cast<const void*>(&k_fused_apply<T, M, V, G, NT, W>);
    case Kind::Fixup: return reinterpret_cast<const void*>(&k_fixup<T, M, V, NT, W>);
    case Kind::TrueResidual:
        if constexpr (sizeof(T) == 8)
            return reinterpret_cast<const void*>(&k_true_residual<M, V, G, NT, W>);
        return nullptr;
    case Kind::Residual64:
        if constexpr (sizeof(T) == 8) {
            if (kJs && js)
                return reinterpret_cast<const void*>(&k_residual64<M, V, G, NT, W, kStepResidual, kJs>);
            return reinterpret_cast<const void*>(&k_residual64<M, V, G, NT, W, kStepResidual, false>);
        }
        return nullptr;
    case Kind::Update64:
        if constexpr (sizeof(T) == 8)
            return reinterpret_cast<const void*>(&k_update64<M, V, NT, W>);
        return nullptr;
    default: return nullptr;
    }
}

template <typename T, int M, bool V, bool G>
const void* main_func_n(Kind kind, bool nt, bool w, bool js, bool cz)
{
    // the nontemporal variants exist only where the hint is used: one
    // 16-byte chunk per lane and vector; one column per wavefront: L = 64
    if constexpr (M * sizeof(T) == 16) {
        if (w) return nt ? main_func_m<T, M, V, G, true, true>(kind, js, cz) : main_func_m<T, M, V, G, false, true>(kind, js, cz);
        return nt ? main_func_m<T, M, V, G, true, false>(kind, js, cz) : main_func_m<T, M, V, G, false, false>(kind, js, cz);
    } else {
        if (w) return main_func_m<T, M, V, G, false, true>(kind, js, cz);
        return main_func_m<T, M, V, G, false, false>(kind, js, cz);
    }
}

template <typename T, int M>
const void* main_func_v(Kind kind, const ColArgs& a, bool nt)
{
    // vector path: whole chunks valid and 16-byte aligned rows and chunks
    const bool vec = (a.g.nz % M == 0) && ((M * sizeof(T)) % 16 == 0) &&
                     ((a.g.nz * sizeof(T)) % 16 == 0);
    const bool w = a.L == kWave;
    const bool js = w && a.g.ny % step_of(kind) == 0;
    if (a.hgeo)
        return vec ? main_func_n<T, M, true, true>(kind, nt, w, js, a.cache_z != 0) : main_func_n<T, M, false, true>(kind, nt, w, js, a.cache_z != 0);
    return vec ? main_func_n<T, M, true, false>(kind, nt, w, js, a.cache_z != 0) : main_func_n<T, M, false, false>(kind, nt, w, js, a.cache_z != 0);
}

template <typename T>
const void* main_func(Kind kind, const ColArgs& a, int64_t batch)
{
    if (kind >= Kind::RbFirst) return rb_func<T>(kind, a, batch);
    if (kind >= Kind::MgPre) return mg_func<T>(kind, a, batch);
    const int M = a.L > 0 ? (a.g.nz + a.L - 1) / a.L : 0;
    int Mp = 1;
    while (Mp < M) Mp <<= 1;
    const bool nt = a.g.n * batch * (int64_t)sizeof(T) >= kStreamBytes && Mp * sizeof(T) == 16;
    switch (Mp) {
    case 1: return main_func_v<T, 1>(kind, a, nt);
    case 2: return main_func_v<T, 2>(kind, a, nt);
    case 4: return main_func_v<T, 4>(kind, a, nt);
    case 8: return main_func_v<T, 8>(kind, a, nt);
    case 16: return main_func_v<T, 16>(kind, a, nt);
    default: return nullptr;
    }
}

}  // namespace

// Kernels dominated by the line solve run with their own launch shape.
static inline bool line_solve_kind(Kind k)
{
    return k == Kind::FusedPrec || k == Kind::FusedPrecFirst || k == Kind::Precond ||
           k == Kind::MgPre ||
           k == Kind::MgPreFused || k == Kind::MgPost || k == Kind::MgPostFinal ||
           k == Kind::MgSmooth || k == Kind::MgSmoothFinal || k >= Kind::RbFirst;
}

template <typename T>
int column_launches(Kind kind, const ColArgs& a0, int64_t batch, KernelLaunch out[2])
{
    ColArgs a = a0;
    if (line_solve_kind(kind)) {
        a.L = a0.L_b;
        a.blocks_per_rhs = a0.bpr_b;
    }
    // kernels that take U tiles per wavefront step: at most one workgroup per
    // U tiles (the partial sums follow the launch's own workgroup count)
    if (const int U = step_of(kind); U > 1 && a.L > 0) {
        const int64_t cols = (int64_t)(kWave / a.L) * (kBlock / kWave);
        const int64_t tiles = (a.g.nh + cols - 1) / cols;
        a.blocks_per_rhs = std::max<int64_t>(1, std::min(a.blocks_per_rhs, (tiles + U - 1) / U));
    }
    a.cache_z = a.g.n * batch * (int64_t)sizeof(T) <= kCacheZBytes ? 1 : 0;
    out[0].func = main_func<T>(kind, a, batch);
    if (!out[0].func) return 0;
    out[0].grid = dim3((unsigned)(a.blocks_per_rhs * batch));
    out[0].block = dim3(kBlock);
    out[0].args = a;
    if (a.red_mode == 0 || !has_finalize(kind)) return 1;
    out[1].func = finalize_func(kind);
    out[1].grid = dim3((unsigned)batch);
    out[1].block = dim3(kFinalThreads);
    out[1].args = a;
    return 2;
}


template <typename T>
hipError_t launch_column_main(Kind kind, const ColArgs& a, int64_t batch, hipStream_t s)
{
    KernelLaunch k[2];
    if (column_launches<T>(kind, a, batch, k) < 1) return hipErrorInvalidValue;
    return issue(k[0], s);
}

template <typename T>
hipError_t launch_column_finalize(Kind kind, const ColArgs& a, int64_t batch, hipStream_t s)
{
    KernelLaunch k[2];
    if (column_launches<T>(kind, a, batch, k) < 2) return hipSuccess;
    return issue(k[1], s);
}

template <typename T>
hipError_t launch_column(Kind kind, const ColArgs& a, int64_t batch, hipStream_t s)
{
    KernelLaunch k[2];
    const int n = column_launches<T>(kind, a, batch, k);
    if (n < 1) return hipErrorInvalidValue;
    for (int i = 0; i < n; ++i) {
        const hipError_t e = issue(k[i], s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace pcg
