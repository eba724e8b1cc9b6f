// Device building blocks of the column kernels (included by kernels.h and
// mg.hip): per-column geometry, column loads and stores, the matrix-free
// stencil and the vertical line solve.
//
//
// Work decomposition.  Vertical columns are contiguous in memory (index
// (i*n_y + j)*n_z + k).  A column is handled by a segment of L lanes of one
// wavefront; lane l of the segment owns the M consecutive levels
// k = l*M .. l*M + M-1 (L*M >= n_z), so a wavefront reads 64/L whole columns
// as one contiguous stretch of memory, each lane with wide vector loads.
// Vertical neighbours across lane boundaries travel by cross-lane shuffles;
// horizontal neighbours are the same M levels of the adjacent columns.
//
// Line solve.  The tridiagonal block of a column depends on the column only
// through its class (how many of its four side faces are Dirichlet), so its
// LU factors l_k, 1/D_k, phi_k are computed once per class on the host.  The
// two substitution sweeps are first-order linear recurrences,
//   forward   w_k = r_k - l_k w_{k-1},
//   backward  z_k = w_k / D_k - phi_k z_{k+1},
// which each lane runs over its own levels and the segment completes with a
// scan of affine maps across lanes -- the sub-structuring of the column
// system into L pieces plus an L-sized interface problem (Sec. 6.1).  The
// scan runs in two levels: within each row of 16 lanes by DPP row shifts
// (register moves, no LDS round trip), then across the rows of a 32- or
// 64-lane segment from the rows' totals read into scalar registers.
// L = 1 is the sequential Thomas algorithm of Sec. 4.2.
//
// Stretched horizontal grids (G = true).  |T| and the face weights
// alpha_{T,T'} come from per-index widths, so every column block differs
// and is factorised in the kernel (as the paper's Thomas sweep recomputes
// its coefficients per column): the scaled pivots delta_k obey the continued
// fraction delta_k = g_k - pi_k / delta_{k-1}, a Moebius map of delta_{k-1}.
// Each lane composes the maps of its levels as a 2x2 matrix, the segment
// scans those matrices across lanes (rescaled by powers of two; within rows
// of 16 lanes, then across rows from the rows' products), and each
// lane then runs the recurrence over its own levels from the pivot entering
// them.
//
// Reductions.  Every workgroup writes its partial sums to a fixed slot; the
// last workgroup to finish (atomic ticket) adds the slots in a fixed order and
// performs the scalar step of Alg. InterleavedPCG on the device, so results
// are bitwise reproducible for a given launch shape and no host round trip is
// needed between kernels.
#pragma once

#include "device_common.h"

namespace pcg {
namespace {

// One step of an inclusive scan of affine maps y -> Q + P y within rows of
// 16 lanes: compose with the map D lanes below (UP) or above; lanes whose
// partner lies outside their segment of L lanes (l: position in it) or row
// keep their map.
template <int D, bool UP, typename T>
__device__ __forceinline__ void scan_step(T& P, T& Q, int l, int L)
{
    const T Pn = dpp_move<UP ? kRowShr + D : kRowShl + D, 1>(P);
    const T Qn = dpp_move<UP ? kRowShr + D : kRowShl + D>(Q);
    // segments of 16 lanes or more are whole rows: the lanes whose partner
    // lies outside the segment are exactly those past the row edge, which
    // already received the identity
    if (L >= 16 || (UP ? l >= D : l + D < L)) {
        Q = P * Qn + Q;
        P = P * Pn;
    }
}

// Forward (UP) or backward carry of the recurrence y -> Q + P y run across a
// segment of L lanes (L a power of two, 1..64, segments aligned to L): the
// value entering this lane's levels from the lanes below (UP) or above it,
// starting from zero at the segment's end.  (P, Q): this lane's map.
template <bool UP, typename T>
__device__ __forceinline__ T segment_carry(T P, T Q, int l, int L)
{
    if (L > 1) scan_step<1, UP>(P, Q, l, L);
    if (L > 2) scan_step<2, UP>(P, Q, l, L);
    if (L > 4) scan_step<4, UP>(P, Q, l, L);
    if (L > 8) scan_step<8, UP>(P, Q, l, L);
    // (P, Q) now composes the lanes from the row's (or segment's) edge to
    // this lane; the neighbour's composition, identity at an edge
    T Px = dpp_move<UP ? kRowShr + 1 : kRowShl + 1, 1>(P);
    T Qx = dpp_move<UP ? kRowShr + 1 : kRowShl + 1>(Q);
    if (L < 16 && (UP ? l == 0 : l == L - 1)) {   // (a row edge for L >= 16)
        Px = T(1);
        Qx = T(0);
    }
    if (L <= 16) return Qx;
    // carry into this lane's row from the other rows of the segment, from
    // the rows' totals (last lane of a row going up, first going down)
    const int row = (threadIdx.x & (kWave - 1)) >> 4;
    T cr;
    if constexpr (UP) {
        const T q0 = read_lane(Q, 15), q1 = read_lane(Q, 31), q2 = read_lane(Q, 47);
        if (L == 32) {
            cr = row == 1 ? q0 : row == 3 ? q2 : T(0);
        } else {
            const T p1 = read_lane(P, 31), p2 = read_lane(P, 47);
            const T c2 = q1 + p1 * q0;
            cr = row == 0 ? T(0) : row == 1 ? q0 : row == 2 ? c2 : q2 + p2 * c2;
        }
    } else {
        const T q1 = read_lane(Q, 16), q2 = read_lane(Q, 32), q3 = read_lane(Q, 48);
        if (L == 32) {
            cr = row == 0 ? q1 : row == 2 ? q3 : T(0);
        } else {
            const T p1 = read_lane(P, 16), p2 = read_lane(P, 32);
            const T c1 = q2 + p2 * q3;
            cr = row == 3 ? T(0) : row == 2 ? q3 : row == 1 ? c1 : q1 + p1 * c1;
        }
    }
    return Qx + Px * cr;
}

// Column indices, and element offsets col * n_z within one right-hand side,
// fit 32 bits: problems have fewer than 2^31 unknowns.
struct Col {
    int32_t idx;
    int32_t im, ip, jm, jp;  // neighbour columns, -1 across a Dirichlet face
    int i, j;                // horizontal position
    int cls;                 // column class: 3 * (#Dirichlet x faces) + #Dirichlet y faces
    double alpha_t;          // alpha_T = sum of alpha_{T,T'}, Dirichlet faces twice
    double area;             // stretched grids: |T| and the face weights alpha_{T,T'}
    double wxm, wxp, wym, wyp;
    bool ok;
};

// Per-column geometry of column (i, j) (Sec. 4.2: |T| and alpha_{T,T'} are
// evaluated once per column).  Dirichlet faces use the half-cell distance,
// i.e. they add 2*alpha_{T,T'} to alpha_T.  ok = false: a column past the
// grid (its lanes still take part in the shuffles; i = j = 0 stand in).
template <bool G = false>
__device__ __forceinline__ Col make_col_ij(const Geom& g, int i, int j, bool ok,
                                           const double* hgeo = nullptr)
{
    Col o;
    o.ok = ok;
    if (!ok) i = j = 0;
    o.i = i;
    o.j = j;
    const int32_t cc = i * g.ny + j;
    o.idx = cc;
    int cx = 0, cy = 0;
    if (i > 0) o.im = cc - g.ny;
    else if (g.per_x) o.im = cc + (g.nx - 1) * g.ny;
    else { o.im = -1; ++cx; }
    if (i < g.nx - 1) o.ip = cc + g.ny;
    else if (g.per_x) o.ip = cc - (g.nx - 1) * g.ny;
    else { o.ip = -1; ++cx; }
    if (j > 0) o.jm = cc - 1;
    else if (g.per_y) o.jm = cc + (g.ny - 1);
    else { o.jm = -1; ++cy; }
    if (j < g.ny - 1) o.jp = cc + 1;
    else if (g.per_y) o.jp = cc - (g.ny - 1);
    else { o.jp = -1; ++cy; }
    o.cls = 3 * cx + cy;
    if constexpr (G) {
        // widths w and reciprocal centre distances m (lower), p (upper) per
        // index; a Dirichlet wall's m or p is 2/w and its neighbour is absent
        const double* hx = hgeo;
        const double* hy = hgeo + 3 * (int64_t)g.nx;
        const double wi = hx[i], wj = hy[j];
        o.area = wi * wj;
        o.wxm = wj * hx[g.nx + i];
        o.wxp = wj * hx[2 * g.nx + i];
        o.wym = wi * hy[g.ny + j];
        o.wyp = wi * hy[2 * g.ny + j];
        o.alpha_t = (o.wxm + o.wxp) + (o.wym + o.wyp);
    } else {
        o.alpha_t = (2 + cx) * g.ax + (2 + cy) * g.ay;
    }
    return o;
}

// The same for column index c (i*n_y + j); the grid has fewer than 2^31
// columns, so the split into (i, j) is a 32-bit division.
template <bool G = false>
__device__ __forceinline__ Col make_col(const Geom& g, int64_t c, const double* hgeo = nullptr)
{
    const bool ok = c < g.nh;
    const uint32_t cc = ok ? (uint32_t)c : 0u;
    const uint32_t i = cc / (uint32_t)g.ny;
    return make_col_ij<G>(g, (int)i, (int)(cc - i * (uint32_t)g.ny), ok, hgeo);
}

// Load / store the M levels k0..k0+M-1 of column `col`.  V: n_z is a
// multiple of M and rows are 16-byte aligned, so whole chunks are valid and
// move as 16-byte vector accesses.  NT: the access carries the nontemporal
// hint (vectors streamed once per kernel, larger than the caches).
template <bool NT, typename T>
__device__ __forceinline__ T ld1(const T* p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <bool NT, typename T>
__device__ __forceinline__ void st1(T* p, T v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// The vector path loads unconditionally (a chunk outside the grid reads
// column 0, a lane past n_z the column's last chunk) and zeroes the result
// by a select: no branch around the load, so the compiler can issue the
// loads of a column and of its neighbours together and wait for them once.
// The column part of the address stays uniform when the column is (one
// column per wavefront), so the loads take a scalar base and a per-lane
// offset.
// Alignment of a lane's chunk of M values in the vector path (whole chunks,
// rows a multiple of the chunk): its size, at most 16 bytes.
template <typename T, int M>
constexpr size_t kChunkAlign = M * sizeof(T) >= 16 ? 16 : M * sizeof(T);

template <typename T, int M, bool V, bool NT = false>
__device__ __forceinline__ void ld(const T* __restrict__ v, int64_t col, bool ok, int k0,
                                   int nz, T (&o)[M])
{
    if (V) {
        const bool in = ok && k0 < nz;
        // the lane's part of the address as a 32-bit byte offset (a column
        // holds < 2^32 bytes): with a uniform column the load then takes a
        // scalar base and one offset register shared by every column
        const uint32_t kb = uint32_t(k0 < nz ? k0 : nz - M) * uint32_t(sizeof(T));
        const T* base = v + uint32_t(ok ? col : int64_t(0)) * uint32_t(nz);
        const T* p = static_cast<const T*>(__builtin_assume_aligned(
            reinterpret_cast<const char*>(base) + kb, kChunkAlign<T, M>));
#pragma unroll
        for (int t = 0; t < M; ++t) o[t] = ld1<NT>(p + t);
#pragma unroll
        for (int t = 0; t < M; ++t) o[t] = in ? o[t] : T(0);
    } else {
#pragma unroll
        for (int t = 0; t < M; ++t) {
            const int k = k0 + t;
            o[t] = (ok && k < nz) ? ld1<NT>(v + col * nz + k) : T(0);
        }
    }
}

template <typename T, int M, bool V, bool NT = false>
__device__ __forceinline__ void st(T* __restrict__ v, int64_t col, bool ok, int k0, int nz,
                                   const T (&o)[M])
{
    if (V) {
        if (ok && k0 < nz) {
            T* base = v + uint32_t(col) * uint32_t(nz);
            T* p = static_cast<T*>(__builtin_assume_aligned(
                reinterpret_cast<char*>(base) + uint32_t(k0) * uint32_t(sizeof(T)),
                kChunkAlign<T, M>));
#pragma unroll
            for (int t = 0; t < M; ++t) st1<NT>(p + t, o[t]);
        }
    } else {
#pragma unroll
        for (int t = 0; t < M; ++t) {
            const int k = k0 + t;
            if (ok && k < nz) st1<NT>(v + col * nz + k, o[t]);
        }
    }
}

// Marks values as computed at this point (an empty statement that uses and
// redefines their registers): a value used only by a store inside the
// store's guard would otherwise be computed, and its load issued, inside
// that guard -- after the tile's other loads had been waited for.
template <typename T, int M>
__device__ __forceinline__ void keep_here(T (&v)[M])
{
#pragma unroll
    for (int i = 0; i < M; ++i) asm volatile("" : "+v"(v[i]));
}

// Level table row `comp` (length nzp, zero-padded), levels k0..k0+M-1.
template <typename T, int M, bool V>
__device__ __forceinline__ void ld_tab(const T* __restrict__ tab, int comp, int nzp, int k0,
                                       int nz, T (&o)[M])
{
    const T* row = tab + (int64_t)comp * nzp;
    if (V) {
        if (k0 < nz) {
            const T* p = static_cast<const T*>(__builtin_assume_aligned(row + k0, 16));
#pragma unroll
            for (int t = 0; t < M; ++t) o[t] = p[t];
        } else {
#pragma unroll
            for (int t = 0; t < M; ++t) o[t] = T(0);
        }
    } else {
#pragma unroll
        for (int t = 0; t < M; ++t) o[t] = (k0 + t < nz) ? row[k0 + t] : T(0);
    }
}

// (A x) on this lane's levels (eq. for the matrix-free product, Sec. 4.2,
// in the unprimed form of eq. TridiagonalMatrix):
//   y_k = |T| [ s_k x_k + b_k x_{k+1} + c_k x_{k-1} ]
//       + d_k [ sum_{T'} alpha_{T,T'} x_{T',k} - alpha_T x_k ],   s = a - b - c.
// xc: this lane's levels of x (zero beyond n_z); x: the whole vector for the
// horizontal neighbours.
// The vertical coefficients of this lane's levels (the same for every column
// a lane visits, so loaded once per kernel).
template <typename T, int M>
struct VertCoef {
    T s[M], b[M], c[M], d[M];
};

template <typename T, int M, bool V>
__device__ __forceinline__ VertCoef<T, M> load_vert(const Geom& g, const T* __restrict__ vert,
                                                    int k0)
{
    VertCoef<T, M> v;
    ld_tab<T, M, V>(vert, 0, g.nzp, k0, g.nz, v.s);
    ld_tab<T, M, V>(vert, 1, g.nzp, k0, g.nz, v.b);
    ld_tab<T, M, V>(vert, 2, g.nzp, k0, g.nz, v.c);
    ld_tab<T, M, V>(vert, 3, g.nzp, k0, g.nz, v.d);
    return v;
}

// The same with the four horizontal neighbours' levels supplied by
// nb(direction, column, valid, out), direction 0..3 for the neighbours
// i-1, i+1, j-1, j+1 (valid = false must give zeros).
template <typename T, int M, bool G, typename NbLoad>
__device__ __forceinline__ void stencil_nb(const Geom& g, const Col& c, int l, int L,
                                           const T (&xc)[M], const VertCoef<T, M>& vc,
                                           NbLoad&& nb, T (&y)[M])
{
    T xim[M], xip[M], xjm[M], xjp[M];
    nb(0, c.im, c.ok && c.im >= 0, xim);
    nb(1, c.ip, c.ok && c.ip >= 0, xip);
    nb(2, c.jm, c.ok && c.jm >= 0, xjm);
    nb(3, c.jp, c.ok && c.jp >= 0, xjp);

    T below = dpp_move<kWaveShr1>(xc[M - 1]);
    T above = dpp_move<kWaveShl1>(xc[0]);
    if (l == 0) below = T(0);
    if (l == L - 1) above = T(0);

    const T at = T(c.alpha_t);
    if constexpr (G) {
        const T area = T(c.area), wxm = T(c.wxm), wxp = T(c.wxp), wym = T(c.wym),
                wyp = T(c.wyp);
#pragma unroll
        for (int t = 0; t < M; ++t) {
            const T lo = t == 0 ? below : xc[t - 1];
            const T hi = t == M - 1 ? above : xc[t + 1];
            const T vertical = area * (vc.s[t] * xc[t] + vc.b[t] * hi + vc.c[t] * lo);
            const T horizontal = vc.d[t] * ((wxm * xim[t] + wxp * xip[t]) +
                                            (wym * xjm[t] + wyp * xjp[t]) - at * xc[t]);
            y[t] = vertical + horizontal;
        }
    } else {
        const T area = T(g.area), ax = T(g.ax), ay = T(g.ay);
#pragma unroll
        for (int t = 0; t < M; ++t) {
            const T lo = t == 0 ? below : xc[t - 1];
            const T hi = t == M - 1 ? above : xc[t + 1];
            const T vertical = area * (vc.s[t] * xc[t] + vc.b[t] * hi + vc.c[t] * lo);
            const T horizontal =
                vc.d[t] * (ax * (xim[t] + xip[t]) + ay * (xjm[t] + xjp[t]) - at * xc[t]);
            y[t] = vertical + horizontal;
        }
    }
}

// A stencil's inputs loaded ahead of its arithmetic: the column's levels and
// the same levels of its four horizontal neighbours (zeros across Dirichlet
// faces).  Loading them first, together with a kernel's other loads, lets
// all of a tile's memory accesses be in flight at once.
template <typename T, int M>
struct StencilIn {
    T xc[M];
    T nb[4][M];
};

template <typename T, int M, bool V>
__device__ __forceinline__ void load_stencil(const Geom& g, const Col& c, int k0,
                                             const T* __restrict__ x, StencilIn<T, M>& in)
{
    ld<T, M, V>(x, c.idx, c.ok, k0, g.nz, in.xc);
    ld<T, M, V>(x, c.im, c.ok && c.im >= 0, k0, g.nz, in.nb[0]);
    ld<T, M, V>(x, c.ip, c.ok && c.ip >= 0, k0, g.nz, in.nb[1]);
    ld<T, M, V>(x, c.jm, c.ok && c.jm >= 0, k0, g.nz, in.nb[2]);
    ld<T, M, V>(x, c.jp, c.ok && c.jp >= 0, k0, g.nz, in.nb[3]);
}

template <typename T, int M, bool G = false>
__device__ __forceinline__ void stencil_in(const Geom& g, const Col& c, int l, int L,
                                           const StencilIn<T, M>& in, const VertCoef<T, M>& vc,
                                           T (&y)[M])
{
    stencil_nb<T, M, G>(g, c, l, L, in.xc, vc,
                        [&](int d, int64_t, bool, T (&o)[M]) {
#pragma unroll
                            for (int t = 0; t < M; ++t) o[t] = in.nb[d][t];
                        },
                        y);
}

template <typename T, int M, bool V, bool G = false>
__device__ __forceinline__ void stencil(const Geom& g, const Col& c, int l, int L, int k0,
                                        const T* __restrict__ x, const T (&xc)[M],
                                        const VertCoef<T, M>& vc, T (&y)[M])
{
    stencil_nb<T, M, G>(g, c, l, L, xc, vc,
                        [&](int, int64_t col, bool ok, T (&o)[M]) {
                            ld<T, M, V>(x, col, ok, k0, g.nz, o);
                        },
                        y);
}

// z = M^{-1} r on one column segment (see the file comment).  r: this
// lane's levels; on return z holds the solution on them.
// LU factors of one column class on this lane's levels.
template <typename T, int M>
struct LuCoef {
    T l[M], inv_d[M], phi[M];
};

template <typename T, int M, bool V>
__device__ __forceinline__ LuCoef<T, M> load_lu(const Geom& g, const T* __restrict__ lu, int cls,
                                                int k0)
{
    LuCoef<T, M> f;
    const T* tab = lu + (int64_t)cls * 3 * g.nzp;
    ld_tab<T, M, V>(tab, 0, g.nzp, k0, g.nz, f.l);
    ld_tab<T, M, V>(tab, 1, g.nzp, k0, g.nz, f.inv_d);
    ld_tab<T, M, V>(tab, 2, g.nzp, k0, g.nz, f.phi);
    return f;
}

// Coefficients of the line solve loaded once per kernel: on uniform grids
// the class-0 factors (interior / periodic columns; columns of another class
// load theirs), on stretched grids the scaled level vectors from which
// every column's factors are computed.
template <typename T, int M, bool G>
struct SolveCoef {
    LuCoef<T, M> f0;
};
template <typename T, int M>
struct SolveCoef<T, M, true> {
    T e[M], pi[M], cs[M], bs[M], is[M];
};

template <typename T, int M, bool V, bool G>
__device__ __forceinline__ SolveCoef<T, M, G> load_solve(const Geom& g, const ColArgs& a, int k0)
{
    SolveCoef<T, M, G> sc;
    if constexpr (G) {
        const T* vert = static_cast<const T*>(a.vert);
        ld_tab<T, M, V>(vert, 4, g.nzp, k0, g.nz, sc.e);
        ld_tab<T, M, V>(vert, 5, g.nzp, k0, g.nz, sc.pi);
        ld_tab<T, M, V>(vert, 6, g.nzp, k0, g.nz, sc.cs);
        ld_tab<T, M, V>(vert, 7, g.nzp, k0, g.nz, sc.bs);
        ld_tab<T, M, V>(vert, 8, g.nzp, k0, g.nz, sc.is);
    } else {
        sc.f0 = load_lu<T, M, V>(g, static_cast<const T*>(a.lu), 0, k0);
    }
    return sc;
}

// Rescale a 2x2 matrix by a power of two so its largest entry lies in
// [1/2, 1) (exact; the matrix acts projectively).
template <typename T>
__device__ __forceinline__ void rescale(T& e00, T& e01, T& e10, T& e11)
{
    const T m = fmax(fmax(fabs(e00), fabs(e01)), fmax(fabs(e10), fabs(e11)));
    int ex;
    (void)frexp(m, &ex);
    e00 = ldexp(e00, -ex);
    e01 = ldexp(e01, -ex);
    e10 = ldexp(e10, -ex);
    e11 = ldexp(e11, -ex);
}

// The same for a vector.
__device__ __forceinline__ void rescale_vec(double& v0, double& v1)
{
    int ex;
    (void)frexp(fmax(fabs(v0), fabs(v1)), &ex);
    v0 = ldexp(v0, -ex);
    v1 = ldexp(v1, -ex);
}

// One step of the within-row scan of 2x2 matrices (later lanes on the left):
// compose with the product D lanes below; lanes whose partner lies below
// their row (identity) or segment keep theirs.
template <int D>
__device__ __forceinline__ void mobius_step(double& e00, double& e01, double& e10, double& e11,
                                            int l)
{
    const double f00 = dpp_move<kRowShr + D, 1>(e00), f01 = dpp_move<kRowShr + D>(e01);
    const double f10 = dpp_move<kRowShr + D>(e10), f11 = dpp_move<kRowShr + D, 1>(e11);
    if (l >= D) {
        const double n00 = e00 * f00 + e01 * f10, n01 = e00 * f01 + e01 * f11;
        const double n10 = e10 * f00 + e11 * f10, n11 = e10 * f01 + e11 * f11;
        e00 = n00;
        e01 = n01;
        e10 = n10;
        e11 = n11;
        rescale(e00, e01, e10, e11);
    }
}

// LU factors of one stretched-grid column on this lane's levels.  Scaled by
// 1/|T| the block is tridiag(c, s - (alpha_T/|T|) d, b); its pivots are
// D_k = s_k delta_k with delta_k = g_k - pi_k / delta_{k-1} (delta_{-1}
// infinite), g_k = 1 + (alpha_T/|T|) e_k.  In homogeneous coordinates (n, m)
// with delta = n/m one level is the matrix [[g_k, -pi_k], [1, 0]].  Then
// l_k = c_k / D_{k-1} = cs_k / delta_{k-1}, 1/(|T| D_k) = is_k / (|T| delta_k)
// and phi_k = b_k / D_k = bs_k / delta_k; levels beyond n_z get zero factors.
// The factorisation runs in FP64 for either precision: composing many
// levels of a strongly coupled column cancels digits (the pivot map is close
// to one with a double fixed point), and FP64 keeps the rounded factors as
// accurate as the host-computed ones of the uniform path.
template <typename T, int M>
__device__ __forceinline__ void gen_factors(const Col& c, int l, int L, int k0, int nz,
                                            const SolveCoef<T, M, true>& sc, LuCoef<T, M>& f)
{
    const double at = c.alpha_t / c.area;
    const double inv_area = 1.0 / c.area;
    double gk[M];
#pragma unroll
    for (int t = 0; t < M; ++t) gk[t] = 1.0 + at * double(sc.e[t]);
    // this lane's levels, composed (later levels on the left)
    double e00 = 1.0, e01 = 0.0, e10 = 0.0, e11 = 1.0;
#pragma unroll
    for (int t = 0; t < M; ++t) {
        if (k0 + t < nz) {
            const double pi = double(sc.pi[t]);
            const double n00 = gk[t] * e00 - pi * e10;
            const double n01 = gk[t] * e01 - pi * e11;
            e10 = e00;
            e11 = e01;
            e00 = n00;
            e01 = n01;
            rescale(e00, e01, e10, e11);
        }
    }
    // inclusive scan within rows of 16 lanes: lane l ends with the product
    // over the lanes from its row's (or segment's) start up to l
    if (L > 1) mobius_step<1>(e00, e01, e10, e11, l);
    if (L > 2) mobius_step<2>(e00, e01, e10, e11, l);
    if (L > 4) mobius_step<4>(e00, e01, e10, e11, l);
    if (L > 8) mobius_step<8>(e00, e01, e10, e11, l);
    // the lanes below this one within its row (identity at a row start) ...
    const double x00 = dpp_move<kRowShr + 1, 1>(e00), x01 = dpp_move<kRowShr + 1>(e01);
    const double x10 = dpp_move<kRowShr + 1>(e10), x11 = dpp_move<kRowShr + 1, 1>(e11);
    // ... applied to what the rows below it in the segment make of
    // delta_{-1} = (1, 0), from the rows' products
    double v0 = 1.0, v1 = 0.0;
    if (L > 16) {
        const int row = (threadIdx.x & (kWave - 1)) >> 4;
        const double a00 = read_lane(e00, 15), a10 = read_lane(e10, 15);
        if (L == 32) {
            const double c00 = read_lane(e00, 47), c10 = read_lane(e10, 47);
            if (row == 1) {
                v0 = a00;
                v1 = a10;
            } else if (row == 3) {
                v0 = c00;
                v1 = c10;
            }
        } else {
            double w0 = read_lane(e00, 31) * a00 + read_lane(e01, 31) * a10;
            double w1 = read_lane(e10, 31) * a00 + read_lane(e11, 31) * a10;
            rescale_vec(w0, w1);
            double y0 = read_lane(e00, 47) * w0 + read_lane(e01, 47) * w1;
            double y1 = read_lane(e10, 47) * w0 + read_lane(e11, 47) * w1;
            rescale_vec(y0, y1);
            if (row == 1) {
                v0 = a00;
                v1 = a10;
            } else if (row == 2) {
                v0 = w0;
                v1 = w1;
            } else if (row == 3) {
                v0 = y0;
                v1 = y1;
            }
        }
    }
    // pivot entering this lane: the lanes below applied to delta_{-1} = (1, 0)
    const double b00 = x00 * v0 + x01 * v1, b10 = x10 * v0 + x11 * v1;
    double inv_prev = l == 0 ? 0.0 : b10 / b00;
#pragma unroll
    for (int t = 0; t < M; ++t) {
        const int k = k0 + t;
        if (k < nz) {
            const double inv = 1.0 / (gk[t] - double(sc.pi[t]) * inv_prev);
            f.l[t] = T(double(sc.cs[t]) * inv_prev);
            f.inv_d[t] = T((double(sc.is[t]) * inv) * inv_area);
            f.phi[t] = T(double(sc.bs[t]) * inv);
            inv_prev = inv;
        } else {
            f.l[t] = T(0);
            f.inv_d[t] = T(0);
            f.phi[t] = T(0);
        }
    }
}

template <typename T, int M, bool V, bool G>
__device__ __forceinline__ void line_solve(const Geom& g, const Col& c, int l, int L, int k0,
                                           const T* __restrict__ lu, const SolveCoef<T, M, G>& sc,
                                           const T (&r)[M], T (&z)[M])
{
    LuCoef<T, M> f;
    if constexpr (G) {
        gen_factors<T, M>(c, l, L, k0, g.nz, sc, f);
    } else {
        f = sc.f0;
        if (c.cls != 0) f = load_lu<T, M, V>(g, lu, c.cls, k0);
    }
    const T (&lf)[M] = f.l;
    const T (&inv_d)[M] = f.inv_d;
    const T (&phi)[M] = f.phi;

    // forward substitution, local part: w = Q + P * w_in
    T P = T(1), Q = T(0);
    T pi[M];
#pragma unroll
    for (int t = 0; t < M; ++t) {
        Q = r[t] - lf[t] * Q;
        P = -lf[t] * P;
        z[t] = Q;
        pi[t] = P;
    }
    T carry = segment_carry<true>(P, Q, l, L);
#pragma unroll
    for (int t = 0; t < M; ++t) z[t] += pi[t] * carry;

    // backward substitution, local part from the top of the lane's levels
    P = T(1);
    Q = T(0);
#pragma unroll
    for (int t = M - 1; t >= 0; --t) {
        Q = z[t] * inv_d[t] - phi[t] * Q;
        P = -phi[t] * P;
        z[t] = Q;
        pi[t] = P;
    }
    carry = segment_carry<false>(P, Q, l, L);
#pragma unroll
    for (int t = 0; t < M; ++t) z[t] += pi[t] * carry;
}

// Tiles (4 waves x 64/L columns each) of this workgroup.
__device__ __forceinline__ void block_tiles(const Geom& g, int L, int64_t blk, int64_t nblk,
                                            int64_t& t0, int64_t& t1)
{
    // tiles and workgroups number < 2^31: 32-bit divisions; the first
    // ntiles mod nblk workgroups take one tile more
    const uint32_t cols = uint32_t(kWave / L) * uint32_t(kBlock / kWave);
    const uint32_t ntiles = (uint32_t(g.nh) + cols - 1) / cols;
    const uint32_t b = uint32_t(blk), nb = uint32_t(nblk);
    const uint32_t q = ntiles / nb, r = ntiles - q * nb;
    t0 = int64_t(b) * q + (b < r ? b : r);
    t1 = t0 + q + (b < r ? 1 : 0);
}

// Right-hand side and workgroup within it of launch workgroup t (grids have
// fewer than 2^31 workgroups: a 32-bit division).
__device__ __forceinline__ void split_rhs(int64_t t, int64_t bpr, int64_t& rhs, int64_t& blk)
{
    const uint32_t r = uint32_t(t) / uint32_t(bpr);
    rhs = r;
    blk = t - int64_t(r) * bpr;
}

struct Lane {
    int l, seg, wave, k0;
};

template <int M>
__device__ __forceinline__ Lane lane_pos(int L)
{
    Lane o;
    const int lane = threadIdx.x & (kWave - 1);
    o.wave = threadIdx.x / kWave;
    o.seg = lane / L;
    o.l = lane - o.seg * L;
    o.k0 = o.l * M;
    return o;
}

__device__ __forceinline__ int64_t tile_col(int64_t tile, const Lane& p, int L)
{
    return (tile * (kBlock / kWave) + p.wave) * (kWave / L) + p.seg;
}

// The same for one column per wavefront (L = 64): the index is the same in
// every lane, so it is made a scalar (and with it the column's geometry and
// the base addresses of its loads and stores).  Columns number < 2^31.
__device__ __forceinline__ int64_t wave_col(int64_t tile, const Lane& p)
{
    return __builtin_amdgcn_readfirstlane((int)(tile * (kBlock / kWave) + p.wave));
}

}  // namespace
}  // namespace pcg
