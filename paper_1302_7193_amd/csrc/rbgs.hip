// Symmetric block Gauss-Seidel preconditioner over vertical columns in
// red-black order (gfx950).
//
// Sec. 4.1 of the paper: block-SOR preconditioners invert the same
// block-diagonal matrix as the line preconditioner plus one more sparse
// matrix-vector product.  With the columns coloured red (i + j even) and
// black, every neighbour of a column has the other colour, and one forward
// plus one backward block Gauss-Seidel sweep from zero is
//   red:   z_R = D^{-1} r_R
//   black: z_B = D^{-1} (r_B - A_BR z_R)
//   red:   z_R = D^{-1} (r_R - A_RB z_B)
// (the backward sweep's black step repeats the forward one).  A_BR, A_RB
// are the horizontal couplings of the stencil; D^{-1} is the line solve.
// Each half-sweep reads only the other colour, so all three write into the
// same vector z.  The first kernel also does kernel B's update of r, the
// last its reductions and scalar step.
// NT: r, q and the stores of z go with the nontemporal hint (the colour read
// through the neighbour loads does not); W: one column per wavefront
// (L = 64, column index scalar), as in the fused kernels.
#include "column.h"

namespace pcg {
namespace {

__device__ __forceinline__ bool is_red(const Col& c) { return ((c.i + c.j) & 1) == 0; }

// Horizontal couplings d_k sum_{T'} alpha_{T,T'} x_{T',k} of column c.
template <typename T, int M, bool V, bool G>
__device__ __forceinline__ void hcouple(const Geom& g, const Col& c, int k0,
                                        const T* __restrict__ x, const VertCoef<T, M>& vc,
                                        T (&h)[M])
{
    T xim[M], xip[M], xjm[M], xjp[M];
    ld<T, M, V>(x, c.im, c.ok && c.im >= 0, k0, g.nz, xim);
    ld<T, M, V>(x, c.ip, c.ok && c.ip >= 0, k0, g.nz, xip);
    ld<T, M, V>(x, c.jm, c.ok && c.jm >= 0, k0, g.nz, xjm);
    ld<T, M, V>(x, c.jp, c.ok && c.jp >= 0, k0, g.nz, xjp);
    if constexpr (G) {
        const T wxm = T(c.wxm), wxp = T(c.wxp), wym = T(c.wym), wyp = T(c.wyp);
#pragma unroll
        for (int t = 0; t < M; ++t)
            h[t] = vc.d[t] * ((wxm * xim[t] + wxp * xip[t]) + (wym * xjm[t] + wyp * xjp[t]));
    } else {
        const T ax = T(g.ax), ay = T(g.ay);
#pragma unroll
        for (int t = 0; t < M; ++t) h[t] = vc.d[t] * (ax * (xim[t] + xip[t]) + ay * (xjm[t] + xjp[t]));
    }
}

// Red columns: z = D^{-1} r.  FUSED: first r -= alpha q on every column (or
// r taken from b in the first iteration), as kernel B does.  Reads r from
// a.in0 (FUSED: a.in1 / a.io1 and q = a.io4, r written to a.io1); writes
// the red columns of z = a.io2.
template <typename T, int M, bool V, bool G, bool FUSED, bool NT, bool W>
__global__ __launch_bounds__(kBlock) void k_rb_first(ColArgs a)
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
    const Lane p = lane_pos<M>(L);
    const SolveCoef<T, M, G> sc = load_solve<T, M, V, G>(g, a, p.k0);
    int64_t t0, t1;
    block_tiles(g, L, blk, a.blocks_per_rhs, t0, t1);
    for (int64_t tile = t0; tile < t1; ++tile) {
        const Col c = make_col<G>(g, W ? wave_col(tile, p) : tile_col(tile, p, L), a.hgeo);
        const bool red = is_red(c);
        T rc[M];
        if constexpr (FUSED) {
            ld<T, M, V, NT>(src, c.idx, c.ok, p.k0, g.nz, rc);
            if (!first) {
                T qc[M];
                ld<T, M, V, NT>(q, c.idx, c.ok, p.k0, g.nz, qc);
#pragma unroll
                for (int i = 0; i < M; ++i) rc[i] = rc[i] - alpha * qc[i];
            }
            if (!first || store_r) st<T, M, V, NT>(r, c.idx, c.ok, p.k0, g.nz, rc);
        } else {
            ld<T, M, V, NT>(src, c.idx, c.ok && red, p.k0, g.nz, rc);
        }
        if (red) {   // the same for every lane of the column's segment
            T zc[M];
            line_solve<T, M, V, G>(g, c, p.l, L, p.k0, lu, sc, rc, zc);
            st<T, M, V, NT>(z, c.idx, c.ok, p.k0, g.nz, zc);
        }
    }
}

// One later half-sweep over the columns of colour RED (reads r = a.in0 and
// the other colour of z = a.io2, writes this colour of z).  FINAL (red):
// R = <r,r>, kappa = <r,z> over all columns, exit test, beta.
// CZ: z stored without the nontemporal hint (ColArgs::cache_z), in the black
// half-sweep and the final red one: kernel A reads z next.
template <typename T, int M, bool V, bool G, bool RED, bool FINAL, bool NT, bool W,
          bool CZ = false>
__global__ __launch_bounds__(kBlock) void k_rb_sweep(ColArgs a)
{
    const Geom& g = a.g;
    const int L = W ? kWave : a.L;
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    int64_t rhs, blk;
    split_rhs(t, a.blocks_per_rhs, rhs, blk);
    SolverState* s = a.st ? a.st + rhs : nullptr;
    if (s && s->flag != kRunning) return;
    const int64_t off = rhs * g.n;
    const T* r = static_cast<const T*>(a.in0) + off;
    T* z = static_cast<T*>(a.io2) + off;
    const T* lu = static_cast<const T*>(a.lu);
    const Lane p = lane_pos<M>(L);
    const VertCoef<T, M> vc = load_vert<T, M, V>(g, static_cast<const T*>(a.vert), p.k0);
    const SolveCoef<T, M, G> sc = load_solve<T, M, V, G>(g, a, p.k0);
    double acc[2] = {0.0, 0.0};
    int64_t t0, t1;
    block_tiles(g, L, blk, a.blocks_per_rhs, t0, t1);
    for (int64_t tile = t0; tile < t1; ++tile) {
        const Col c = make_col<G>(g, W ? wave_col(tile, p) : tile_col(tile, p, L), a.hgeo);
        const bool mine = is_red(c) == RED;
        if (!mine && !FINAL) continue;   // the same for every lane of the segment
        T rc[M], zc[M];
        ld<T, M, V, NT>(r, c.idx, c.ok, p.k0, g.nz, rc);
        if (mine) {
            T h[M];
            hcouple<T, M, V, G>(g, c, p.k0, z, vc, h);
#pragma unroll
            for (int i = 0; i < M; ++i) h[i] = rc[i] - h[i];
            line_solve<T, M, V, G>(g, c, p.l, L, p.k0, lu, sc, h, zc);
            st<T, M, V, NT && !CZ>(z, c.idx, c.ok, p.k0, g.nz, zc);
        } else {
            ld<T, M, V>(z, c.idx, c.ok, p.k0, g.nz, zc);
        }
        if constexpr (FINAL) {
#pragma unroll
            for (int i = 0; i < M; ++i) {
                acc[0] += double(rc[i]) * double(rc[i]);
                acc[1] += double(rc[i]) * double(zc[i]);
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
const void* rb_func_m(Kind kind, bool cz)
{
    switch (kind) {
    case Kind::RbFirst:
        return reinterpret_cast<const void*>(&k_rb_first<T, M, V, G, false, NT, W>);
    case Kind::RbFirstFused:
        return reinterpret_cast<const void*>(&k_rb_first<T, M, V, G, true, NT, W>);
    case Kind::RbBlack:
        if (NT && cz) return reinterpret_cast<const void*>(&k_rb_sweep<T, M, V, G, false, false, NT, W, true>);
        return reinterpret_cast<const void*>(&k_rb_sweep<T, M, V, G, false, false, NT, W>);
    case Kind::RbRed:
        return reinterpret_cast<const void*>(&k_rb_sweep<T, M, V, G, true, false, NT, W>);
    case Kind::RbRedFinal:
        if (NT && cz) return reinterpret_cast<const void*>(&k_rb_sweep<T, M, V, G, true, true, NT, W, true>);
        return reinterpret_cast<const void*>(&k_rb_sweep<T, M, V, G, true, true, NT, W>);
    default: return nullptr;
    }
}

template <typename T, int M, bool V, bool G>
const void* rb_func_n(Kind kind, bool nt, bool w, bool cz)
{
    // the nontemporal variants exist only where the hint is used: one
    // 16-byte chunk per lane and vector
    if constexpr (M * sizeof(T) == 16) {
        if (w) return nt ? rb_func_m<T, M, V, G, true, true>(kind, cz) : rb_func_m<T, M, V, G, false, true>(kind, cz);
        return nt ? rb_func_m<T, M, V, G, true, false>(kind, cz) : rb_func_m<T, M, V, G, false, false>(kind, cz);
    } else {
        return w ? rb_func_m<T, M, V, G, false, true>(kind, cz) : rb_func_m<T, M, V, G, false, false>(kind, cz);
    }
}

template <typename T, int M>
const void* rb_func_v(Kind kind, const ColArgs& a, bool nt)
{
    const bool vec = (a.g.nz % M == 0) && ((M * sizeof(T)) % 16 == 0) &&
                     ((a.g.nz * sizeof(T)) % 16 == 0);
    const bool w = a.L == kWave;
    if (a.hgeo) return vec ? rb_func_n<T, M, true, true>(kind, nt, w, a.cache_z != 0) : rb_func_n<T, M, false, true>(kind, nt, w, a.cache_z != 0);
    return vec ? rb_func_n<T, M, true, false>(kind, nt, w, a.cache_z != 0) : rb_func_n<T, M, false, false>(kind, nt, w, a.cache_z != 0);
}

}  // namespace

template <typename T>
const void* rb_func(Kind kind, const ColArgs& a, int64_t batch)
{
    const int M = a.L > 0 ? (a.g.nz + a.L - 1) / a.L : 0;
    int Mp = 1;
    while (Mp < M) Mp <<= 1;
    const bool nt = a.g.n * batch * (int64_t)sizeof(T) >= kStreamBytes && Mp * sizeof(T) == 16;
    switch (Mp) {
    case 1: return rb_func_v<T, 1>(kind, a, nt);
    case 2: return rb_func_v<T, 2>(kind, a, nt);
    case 4: return rb_func_v<T, 4>(kind, a, nt);
    case 8: return rb_func_v<T, 8>(kind, a, nt);
    case 16: return rb_func_v<T, 16>(kind, a, nt);
    default: return nullptr;
    }
}

template const void* rb_func<double>(Kind, const ColArgs&, int64_t);
template const void* rb_func<float>(Kind, const ColArgs&, int64_t);

}  // namespace pcg
