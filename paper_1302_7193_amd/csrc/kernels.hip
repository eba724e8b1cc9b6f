// Column kernels of the line-preconditioned CG solver (gfx950).
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
// log2(L)-step scan of affine maps across lanes -- the sub-structuring of the
// column system into L pieces plus an L-sized interface problem (Sec. 6.1).
// L = 1 is the sequential Thomas algorithm of Sec. 4.2.
//
// Stretched horizontal grids (G = true).  |T| and the face weights
// alpha_{T,T'} come from per-index widths, so every column block differs
// and is factorised in the kernel (as the paper's Thomas sweep recomputes
// its coefficients per column): the scaled pivots delta_k obey the continued
// fraction delta_k = g_k - pi_k / delta_{k-1}, a Moebius map of delta_{k-1}.
// Each lane composes the maps of its levels as a 2x2 matrix, the segment
// scans those matrices across lanes (rescaled by powers of two), and each
// lane then runs the recurrence over its own levels from the pivot entering
// them.
//
// Reductions.  Every workgroup writes its partial sums to a fixed slot; the
// last workgroup to finish (atomic ticket) adds the slots in a fixed order and
// performs the scalar step of Alg. InterleavedPCG on the device, so results
// are bitwise reproducible for a given launch shape and no host round trip is
// needed between kernels.
#include "device_common.h"

namespace pcg {
namespace {

struct Col {
    int64_t idx;
    int64_t im, ip, jm, jp;  // neighbour columns, -1 across a Dirichlet face
    int cls;                 // column class: 3 * (#Dirichlet x faces) + #Dirichlet y faces
    double alpha_t;          // alpha_T = sum of alpha_{T,T'}, Dirichlet faces twice
    double area;             // stretched grids: |T| and the face weights alpha_{T,T'}
    double wxm, wxp, wym, wyp;
    bool ok;
};

// Per-column geometry, recomputed from (i, j) (Sec. 4.2: |T| and
// alpha_{T,T'} are evaluated once per column).  Dirichlet faces use the
// half-cell distance, i.e. they add 2*alpha_{T,T'} to alpha_T.
template <bool G = false>
__device__ __forceinline__ Col make_col(const Geom& g, int64_t c, const double* hgeo = nullptr)
{
    Col o;
    o.ok = c < g.nh;
    const int64_t cc = o.ok ? c : 0;
    o.idx = cc;
    const int64_t i = cc / g.ny, j = cc - i * g.ny;
    int cx = 0, cy = 0;
    if (i > 0) o.im = cc - g.ny;
    else if (g.per_x) o.im = cc + (int64_t)(g.nx - 1) * g.ny;
    else { o.im = -1; ++cx; }
    if (i < g.nx - 1) o.ip = cc + g.ny;
    else if (g.per_x) o.ip = cc - (int64_t)(g.nx - 1) * g.ny;
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

template <typename T, int M, bool V, bool NT = false>
__device__ __forceinline__ void ld(const T* __restrict__ v, int64_t col, bool ok, int k0,
                                   int nz, T (&o)[M])
{
    if (V) {
        if (ok && k0 < nz) {
            const T* p = static_cast<const T*>(__builtin_assume_aligned(v + col * nz + k0, 16));
#pragma unroll
            for (int t = 0; t < M; ++t) o[t] = ld1<NT>(p + t);
        } else {
#pragma unroll
            for (int t = 0; t < M; ++t) o[t] = T(0);
        }
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
            T* p = static_cast<T*>(__builtin_assume_aligned(v + col * nz + k0, 16));
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

template <typename T, int M, bool V, bool G = false>
__device__ __forceinline__ void stencil(const Geom& g, const Col& c, int l, int L, int k0,
                                        const T* __restrict__ x, const T (&xc)[M],
                                        const VertCoef<T, M>& vc, T (&y)[M])
{
    T below = __shfl_up(xc[M - 1], 1, L);
    T above = __shfl_down(xc[0], 1, L);
    if (l == 0) below = T(0);
    if (l == L - 1) above = T(0);

    T xim[M], xip[M], xjm[M], xjp[M];
    ld<T, M, V>(x, c.im, c.ok && c.im >= 0, k0, g.nz, xim);
    ld<T, M, V>(x, c.ip, c.ok && c.ip >= 0, k0, g.nz, xip);
    ld<T, M, V>(x, c.jm, c.ok && c.jm >= 0, k0, g.nz, xjm);
    ld<T, M, V>(x, c.jp, c.ok && c.jp >= 0, k0, g.nz, xjp);

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
    // inclusive scan across the segment: lane l ends with the product over
    // lanes l, l-1, ..., 0
    for (int d = 1; d < L; d <<= 1) {
        const double f00 = __shfl_up(e00, d, L), f01 = __shfl_up(e01, d, L);
        const double f10 = __shfl_up(e10, d, L), f11 = __shfl_up(e11, d, L);
        if (l >= d) {
            const double n00 = e00 * f00 + e01 * f10, n01 = e00 * f01 + e01 * f11;
            const double n10 = e10 * f00 + e11 * f10, n11 = e10 * f01 + e11 * f11;
            e00 = n00;
            e01 = n01;
            e10 = n10;
            e11 = n11;
            rescale(e00, e01, e10, e11);
        }
    }
    // pivot entering this lane: the lanes below applied to delta_{-1} = (1, 0)
    const double b00 = __shfl_up(e00, 1, L), b10 = __shfl_up(e10, 1, L);
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
    for (int d = 1; d < L; d <<= 1) {   // inclusive scan of (P, Q) across the segment
        const T Pp = __shfl_up(P, d, L);
        const T Qp = __shfl_up(Q, d, L);
        if (l >= d) {
            Q = P * Qp + Q;
            P = P * Pp;
        }
    }
    T carry = __shfl_up(Q, 1, L);
    if (l == 0) carry = T(0);
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
    for (int d = 1; d < L; d <<= 1) {   // reverse scan across the segment
        const T Pn = __shfl_down(P, d, L);
        const T Qn = __shfl_down(Q, d, L);
        if (l + d < L) {
            Q = P * Qn + Q;
            P = P * Pn;
        }
    }
    carry = __shfl_down(Q, 1, L);
    if (l == L - 1) carry = T(0);
#pragma unroll
    for (int t = 0; t < M; ++t) z[t] += pi[t] * carry;
}

// Tiles (4 waves x 64/L columns each) of this workgroup.
__device__ __forceinline__ void block_tiles(const Geom& g, int L, int64_t blk, int64_t nblk,
                                            int64_t& t0, int64_t& t1)
{
    const int64_t cols = (int64_t)(kWave / L) * (kBlock / kWave);
    const int64_t ntiles = (g.nh + cols - 1) / cols;
    t0 = blk * ntiles / nblk;
    t1 = (blk + 1) * ntiles / nblk;
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

// ---------------------------------------------------------------- kernels --

template <typename T, int M, bool V, bool G>
__global__ __launch_bounds__(kBlock) void k_apply(ColArgs a)
{
    const Geom& g = a.g;
    const int L = a.L;
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t rhs = t / a.blocks_per_rhs, blk = t - rhs * a.blocks_per_rhs;
    if (a.st && a.st[rhs].flag != kRunning) return;   // inside a solve: stop when done
    const T* x = static_cast<const T*>(a.in0) + rhs * g.n;
    T* y = static_cast<T*>(a.io0) + rhs * g.n;
    const T* vert = static_cast<const T*>(a.vert);
    const Lane p = lane_pos<M>(L);
    const VertCoef<T, M> vc = load_vert<T, M, V>(g, vert, p.k0);
    int64_t t0, t1;
    block_tiles(g, L, blk, a.blocks_per_rhs, t0, t1);
    for (int64_t tile = t0; tile < t1; ++tile) {
        const Col c = make_col<G>(g, tile_col(tile, p, L), a.hgeo);
        T xc[M], yc[M];
        ld<T, M, V>(x, c.idx, c.ok, p.k0, g.nz, xc);
        stencil<T, M, V, G>(g, c, p.l, L, p.k0, x, xc, vc, yc);
        st<T, M, V>(y, c.idx, c.ok, p.k0, g.nz, yc);
    }
}

template <typename T, int M, bool V, bool G>
__global__ __launch_bounds__(kBlock) void k_precond(ColArgs a)
{
    const Geom& g = a.g;
    const int L = a.L;
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t rhs = t / a.blocks_per_rhs, blk = t - rhs * a.blocks_per_rhs;
    if (a.st && a.st[rhs].flag != kRunning) return;
    const T* r = static_cast<const T*>(a.in0) + rhs * g.n;
    T* z = static_cast<T*>(a.io0) + rhs * g.n;
    const T* lu = static_cast<const T*>(a.lu);
    const Lane p = lane_pos<M>(L);
    const SolveCoef<T, M, G> sc = load_solve<T, M, V, G>(g, a, p.k0);
    int64_t t0, t1;
    block_tiles(g, L, blk, a.blocks_per_rhs, t0, t1);
    for (int64_t tile = t0; tile < t1; ++tile) {
        const Col c = make_col<G>(g, tile_col(tile, p, L), a.hgeo);
        T rc[M], zc[M];
        ld<T, M, V>(r, c.idx, c.ok, p.k0, g.nz, rc);
        line_solve<T, M, V, G>(g, c, p.l, L, p.k0, lu, sc, rc, zc);
        st<T, M, V>(z, c.idx, c.ok, p.k0, g.nz, zc);
    }
}

// r = b - A x; ZERO: x = 0, r = b (nothing to copy when b is r), p = q = 0.
template <typename T, int M, bool V, bool ZERO, bool G>
__global__ __launch_bounds__(kBlock) void k_init(ColArgs a)
{
    const Geom& g = a.g;
    const int L = a.L;
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t rhs = t / a.blocks_per_rhs, blk = t - rhs * a.blocks_per_rhs;
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
        const Col c = make_col<G>(g, tile_col(tile, p, L), a.hgeo);
        if (ZERO) {
            st<T, M, V>(x, c.idx, c.ok, p.k0, g.nz, zero);
            if (!in_place) {
                T bc[M];
                ld<T, M, V>(b, c.idx, c.ok, p.k0, g.nz, bc);
                st<T, M, V>(r, c.idx, c.ok, p.k0, g.nz, bc);
            }
        } else {
            T bc[M], rc[M], xc[M], ax[M];
            ld<T, M, V>(b, c.idx, c.ok, p.k0, g.nz, bc);
            ld<T, M, V>(x, c.idx, c.ok, p.k0, g.nz, xc);
            stencil<T, M, V, G>(g, c, p.l, L, p.k0, x, xc, vc, ax);
#pragma unroll
            for (int i = 0; i < M; ++i) rc[i] = bc[i] - ax[i];
            st<T, M, V>(r, c.idx, c.ok, p.k0, g.nz, rc);
        }
        if (ZERO) {   // the unfused iteration reads p and q; the fused one does not
            st<T, M, V>(pp, c.idx, c.ok, p.k0, g.nz, zero);
            st<T, M, V>(q, c.idx, c.ok, p.k0, g.nz, zero);
        }
    }
}

// Kernel B (Alg. InterleavedPrec): r -= alpha q; z = M^{-1} r;
// R = <r,r>, kappa = <r,z> (FP64 accumulation); scalar step: exit test, beta.
// FIRST (no iteration done yet): alpha = 0 and q is unset, so q is not read;
// with a zero start r is taken from b (no start-up kernel), and not stored
// when b is r itself.
template <typename T, int M, bool V, bool FIRST, bool G, bool NT>
__device__ __forceinline__ void fused_prec_body(const ColArgs& a, SolverState* s, int64_t rhs,
                                                int64_t blk, double (&acc)[2])
{
    const Geom& g = a.g;
    const int L = a.L;
    const int64_t off = rhs * g.n;
    const bool from_b = FIRST && s->zero_start;
    const T* src = static_cast<const T*>(from_b ? a.in1 : a.io1) + off;
    T* r = static_cast<T*>(a.io1) + off;
    const bool store_r = !(from_b && a.in1 == a.io1);
    T* z = static_cast<T*>(a.io2) + off;
    const T* q = static_cast<const T*>(a.io4) + off;
    const T* lu = static_cast<const T*>(a.lu);
    const T alpha = T(s->alpha);
    const Lane p = lane_pos<M>(L);
    const SolveCoef<T, M, G> sc = load_solve<T, M, V, G>(g, a, p.k0);
    int64_t t0, t1;
    block_tiles(g, L, blk, a.blocks_per_rhs, t0, t1);
    for (int64_t tile = t0; tile < t1; ++tile) {
        const Col c = make_col<G>(g, tile_col(tile, p, L), a.hgeo);
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
        if (!FIRST || store_r) st<T, M, V, NT>(r, c.idx, c.ok, p.k0, g.nz, rc);
        line_solve<T, M, V, G>(g, c, p.l, L, p.k0, lu, sc, rc, zc);
#pragma unroll
        for (int i = 0; i < M; ++i) acc[1] += double(rc[i]) * double(zc[i]);
        st<T, M, V, NT>(z, c.idx, c.ok, p.k0, g.nz, zc);
    }
}

template <typename T, int M, bool V, bool G, bool NT>
__global__ __launch_bounds__(kBlock) void k_fused_prec(ColArgs a)
{
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t rhs = t / a.blocks_per_rhs, blk = t - rhs * a.blocks_per_rhs;
    SolverState* s = a.st + rhs;
    if (s->flag != kRunning) return;
    double acc[2] = {0.0, 0.0};
    if (s->iter == 0) fused_prec_body<T, M, V, true, G, NT>(a, s, rhs, blk, acc);
    else fused_prec_body<T, M, V, false, G, NT>(a, s, rhs, blk, acc);
    double tot[2];
    if (publish<2>(acc, a.part + rhs * a.blocks_per_rhs * kRedSlots, blk, a.blocks_per_rhs,
                   &s->ticket, a.red_mode, tot)) {
        if (threadIdx.x == 0) finish_prec(s, tot[0], tot[1]);
    }
}

// Kernel A (Alg. InterleavedApply): u += alpha p; p = z + beta p;
// q = A z + beta q; sigma = <p,q> (FP64); scalar step: alpha.
// FIRST: alpha = 0 and p = q = 0, so p = z, q = A z, and u keeps x0 (written
// as zero for a zero start); u, p and q are not read.
template <typename T, int M, bool V, bool FIRST, bool G, bool NT>
__device__ __forceinline__ void fused_apply_body(const ColArgs& a, SolverState* s, int64_t rhs,
                                                 int64_t blk, double (&acc)[1])
{
    const Geom& g = a.g;
    const int L = a.L;
    const int64_t off = rhs * g.n;
    T* u = static_cast<T*>(a.io0) + off;
    const T* z = static_cast<const T*>(a.io2) + off;
    T* pp = static_cast<T*>(a.io3) + off;
    T* q = static_cast<T*>(a.io4) + off;
    const T* vert = static_cast<const T*>(a.vert);
    const T alpha = T(s->alpha), beta = T(s->beta);
    const bool zero_u = FIRST && s->zero_start;
    const Lane p = lane_pos<M>(L);
    const VertCoef<T, M> vc = load_vert<T, M, V>(g, vert, p.k0);
    int64_t t0, t1;
    block_tiles(g, L, blk, a.blocks_per_rhs, t0, t1);
    for (int64_t tile = t0; tile < t1; ++tile) {
        const Col c = make_col<G>(g, tile_col(tile, p, L), a.hgeo);
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
            if (zero_u) {
                T zero[M];
#pragma unroll
                for (int i = 0; i < M; ++i) zero[i] = T(0);
                st<T, M, V, NT>(u, c.idx, c.ok, p.k0, g.nz, zero);
            }
        } else {
            T uc[M];
            ld<T, M, V, NT>(u, c.idx, c.ok, p.k0, g.nz, uc);
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
        st<T, M, V, NT>(pp, c.idx, c.ok, p.k0, g.nz, pc);
        st<T, M, V, NT>(q, c.idx, c.ok, p.k0, g.nz, qc);
    }
}

template <typename T, int M, bool V, bool G, bool NT>
__global__ __launch_bounds__(kBlock) void k_fused_apply(ColArgs a)
{
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t rhs = t / a.blocks_per_rhs, blk = t - rhs * a.blocks_per_rhs;
    SolverState* s = a.st + rhs;
    if (s->flag != kRunning) return;
    double acc[1] = {0.0};
    if (s->iter == 0) fused_apply_body<T, M, V, true, G, NT>(a, s, rhs, blk, acc);
    else fused_apply_body<T, M, V, false, G, NT>(a, s, rhs, blk, acc);
    double tot[1];
    if (publish<1>(acc, a.part + rhs * a.blocks_per_rhs * kRedSlots, blk, a.blocks_per_rhs,
                   &s->ticket, a.red_mode, tot)) {
        if (threadIdx.x == 0) finish_apply(s, tot[0]);
    }
}

// Exit correction u += alpha p (the fused iteration leaves u one step
// behind r).  Runs once: the last workgroup (or the finalize launch) marks
// it done.
template <typename T, int M, bool V, bool NT>
__global__ __launch_bounds__(kBlock) void k_fixup(ColArgs a)
{
    const Geom& g = a.g;
    const int L = a.L;
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t rhs = t / a.blocks_per_rhs, blk = t - rhs * a.blocks_per_rhs;
    SolverState* s = a.st + rhs;
    // stopped before the first iteration: x = x0 (zero for a zero start, which
    // nothing has written yet -- also after a breakdown in the first kernel)
    const bool none = s->iter == 0;
    const bool stopped = s->flag == kConverged || s->flag == kMaxIter ||
                         (s->flag == kBreakdown && none);
    if (!stopped || s->fixed) return;
    if (none && !s->zero_start) return;
    const int64_t off = rhs * g.n;
    T* u = static_cast<T*>(a.io0) + off;
    const T* pp = static_cast<const T*>(a.io3) + off;
    const T alpha = T(s->alpha);
    const Lane p = lane_pos<M>(L);
    int64_t t0, t1;
    block_tiles(g, L, blk, a.blocks_per_rhs, t0, t1);
    for (int64_t tile = t0; tile < t1; ++tile) {
        const Col c = make_col(g, tile_col(tile, p, L));
        T uc[M];
        if (none) {
#pragma unroll
            for (int i = 0; i < M; ++i) uc[i] = T(0);
        } else {
            T pc[M];
            ld<T, M, V, NT>(u, c.idx, c.ok, p.k0, g.nz, uc);
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

// FP64 true residual: ||b - A x|| into state.aux (T = double only).
template <int M, bool V, bool G>
__global__ __launch_bounds__(kBlock) void k_true_residual(ColArgs a)
{
    const Geom& g = a.g;
    const int L = a.L;
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t rhs = t / a.blocks_per_rhs, blk = t - rhs * a.blocks_per_rhs;
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
        const Col c = make_col<G>(g, tile_col(tile, p, L), a.hgeo);
        double xc[M], ax[M], bc[M];
        ld<double, M, V>(x, c.idx, c.ok, p.k0, g.nz, xc);
        ld<double, M, V>(b, c.idx, c.ok, p.k0, g.nz, bc);
        stencil<double, M, V, G>(g, c, p.l, L, p.k0, x, xc, vc, ax);
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

// Refinement residual: r64 = b - A x in FP64 (r64 = b when a.x0_zero),
// ||r64|| into state.rnorm (state.r0norm on the first call), FP32 copy
// r32 = r64 * scale.
template <int M, bool V, bool G>
__global__ __launch_bounds__(kBlock) void k_residual64(ColArgs a)
{
    const Geom& g = a.g;
    const int L = a.L;
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t rhs = t / a.blocks_per_rhs, blk = t - rhs * a.blocks_per_rhs;
    SolverState* s = a.st + rhs;
    if (s->flag != kRunning) return;
    const double* x = static_cast<const double*>(a.in0) + rhs * g.n;
    const double* b = static_cast<const double*>(a.in1) + rhs * g.n;
    float* r32 = static_cast<float*>(a.out32) + rhs * g.n;
    const double* vert = static_cast<const double*>(a.vert);
    const double scale = s->aux;
    const Lane p = lane_pos<M>(L);
    const VertCoef<double, M> vc = load_vert<double, M, V>(g, vert, p.k0);
    int64_t t0, t1;
    block_tiles(g, L, blk, a.blocks_per_rhs, t0, t1);
    double acc[1] = {0.0};
    for (int64_t tile = t0; tile < t1; ++tile) {
        const Col c = make_col<G>(g, tile_col(tile, p, L), a.hgeo);
        double xc[M], ax[M], bc[M];
        float rc[M];
        ld<double, M, V>(b, c.idx, c.ok, p.k0, g.nz, bc);
        if (a.x0_zero) {
#pragma unroll
            for (int i = 0; i < M; ++i) ax[i] = 0.0;
        } else {
            ld<double, M, V>(x, c.idx, c.ok, p.k0, g.nz, xc);
            stencil<double, M, V, G>(g, c, p.l, L, p.k0, x, xc, vc, ax);
        }
#pragma unroll
        for (int i = 0; i < M; ++i) {
            const double d = bc[i] - ax[i];
            acc[0] += d * d;
            rc[i] = float(d * scale);
        }
        // FP32 rows are 16-byte aligned only when M*4 is a multiple of 16
        st<float, M, (V && (M % 4 == 0))>(r32, c.idx, c.ok, p.k0, g.nz, rc);
    }
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

// Refinement update: x64 += (1/scale) * u32, u32 being the inner solution
// (x64 = u32 / scale when a.x0_zero: x is not read).
template <int M, bool V>
__global__ __launch_bounds__(kBlock) void k_update64(ColArgs a)
{
    const Geom& g = a.g;
    const int L = a.L;
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t rhs = t / a.blocks_per_rhs, blk = t - rhs * a.blocks_per_rhs;
    SolverState* s = a.st + rhs;
    if (s->flag != kRunning) return;
    double* x = static_cast<double*>(a.io0) + rhs * g.n;
    const float* u32 = static_cast<const float*>(a.out32) + rhs * g.n;
    const double inv_scale = 1.0 / s->aux;
    const Lane p = lane_pos<M>(L);
    int64_t t0, t1;
    block_tiles(g, L, blk, a.blocks_per_rhs, t0, t1);
    for (int64_t tile = t0; tile < t1; ++tile) {
        const Col c = make_col(g, tile_col(tile, p, L));
        double xc[M];
        float uc[M];
        if (a.x0_zero) {
#pragma unroll
            for (int i = 0; i < M; ++i) xc[i] = 0.0;
        } else {
            ld<double, M, V>(x, c.idx, c.ok, p.k0, g.nz, xc);
        }
        ld<float, M, (V && (M % 4 == 0))>(u32, c.idx, c.ok, p.k0, g.nz, uc);
#pragma unroll
        for (int i = 0; i < M; ++i) xc[i] += inv_scale * double(uc[i]);
        st<double, M, V>(x, c.idx, c.ok, p.k0, g.nz, xc);
    }
}

// Mode-1 reductions: one workgroup per right-hand side totals the published
// partial sums in the same order as mode 0 and performs the scalar step.
template <Kind K>
__global__ __launch_bounds__(kFinalThreads) void k_finalize(ColArgs a)
{
    const int64_t rhs = blockIdx.x;
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

bool has_finalize(Kind k)
{
    return k == Kind::FusedPrec || k == Kind::FusedApply || k == Kind::Fixup ||
           k == Kind::TrueResidual || k == Kind::Residual64;
}

const void* finalize_func(Kind kind)
{
    switch (kind) {
    case Kind::FusedPrec: return reinterpret_cast<const void*>(&k_finalize<Kind::FusedPrec>);
    case Kind::FusedApply: return reinterpret_cast<const void*>(&k_finalize<Kind::FusedApply>);
    case Kind::Fixup: return reinterpret_cast<const void*>(&k_finalize<Kind::Fixup>);
    case Kind::TrueResidual: return reinterpret_cast<const void*>(&k_finalize<Kind::TrueResidual>);
    case Kind::Residual64: return reinterpret_cast<const void*>(&k_finalize<Kind::Residual64>);
    default: return nullptr;
    }
}

template <typename T, int M, bool V, bool G, bool NT>
const void* main_func_m(Kind kind)
{
    switch (kind) {
    case Kind::Apply: return reinterpret_cast<const void*>(&k_apply<T, M, V, G>);
    case Kind::Precond: return reinterpret_cast<const void*>(&k_precond<T, M, V, G>);
    case Kind::InitFull: return reinterpret_cast<const void*>(&k_init<T, M, V, false, G>);
    case Kind::InitZero: return reinterpret_cast<const void*>(&k_init<T, M, V, true, false>);
    case Kind::FusedPrec: return reinterpret_cast<const void*>(&k_fused_prec<T, M, V, G, NT>);
    case Kind::FusedApply: return reinterpret_cast<const void*>(&k_fused_apply<T, M, V, G, NT>);
    case Kind::Fixup: return reinterpret_cast<const void*>(&k_fixup<T, M, V, NT>);
    case Kind::TrueResidual:
        if constexpr (sizeof(T) == 8)
            return reinterpret_cast<const void*>(&k_true_residual<M, V, G>);
        return nullptr;
    case Kind::Residual64:
        if constexpr (sizeof(T) == 8) return reinterpret_cast<const void*>(&k_residual64<M, V, G>);
        return nullptr;
    case Kind::Update64:
        if constexpr (sizeof(T) == 8) return reinterpret_cast<const void*>(&k_update64<M, V>);
        return nullptr;
    }
    return nullptr;
}

template <typename T, int M, bool V, bool G>
const void* main_func_n(Kind kind, bool nt)
{
    return nt ? main_func_m<T, M, V, G, true>(kind) : main_func_m<T, M, V, G, false>(kind);
}

template <typename T, int M>
const void* main_func_v(Kind kind, const ColArgs& a, bool nt)
{
    // vector path: whole chunks valid and 16-byte aligned rows and chunks
    const bool vec = (a.g.nz % M == 0) && ((M * sizeof(T)) % 16 == 0) &&
                     ((a.g.nz * sizeof(T)) % 16 == 0);
    if (a.hgeo)
        return vec ? main_func_n<T, M, true, true>(kind, nt) : main_func_n<T, M, false, true>(kind, nt);
    return vec ? main_func_n<T, M, true, false>(kind, nt) : main_func_n<T, M, false, false>(kind, nt);
}

// Vectors of the fused iteration larger than this are streamed with the
// nontemporal hint: they cannot stay in the caches (32 MB of L2, 256 MB of
// Infinity Cache) from one kernel to the next.  Only when a lane moves one
// 16-byte chunk per vector, so that every store instruction of a wavefront
// covers whole cache lines: with two or more chunks per lane each
// instruction writes every other chunk, and nontemporal stores of such
// partial lines raised the measured write traffic by a tenth.
constexpr int64_t kStreamBytes = int64_t(64) << 20;

template <typename T>
const void* main_func(Kind kind, const ColArgs& a, int64_t batch)
{
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
static bool line_solve_kind(Kind k) { return k == Kind::FusedPrec || k == Kind::Precond; }

template <typename T>
int column_launches(Kind kind, const ColArgs& a0, int64_t batch, KernelLaunch out[2])
{
    ColArgs a = a0;
    if (line_solve_kind(kind)) {
        a.L = a0.L_b;
        a.blocks_per_rhs = a0.bpr_b;
    }
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

hipError_t issue(const KernelLaunch& k, hipStream_t s)
{
    void* args[] = {const_cast<ColArgs*>(&k.args)};
    return hipLaunchKernel(k.func, k.grid, k.block, args, 0, s);
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

template int column_launches<double>(Kind, const ColArgs&, int64_t, KernelLaunch*);
template int column_launches<float>(Kind, const ColArgs&, int64_t, KernelLaunch*);
template hipError_t launch_column<double>(Kind, const ColArgs&, int64_t, hipStream_t);
template hipError_t launch_column<float>(Kind, const ColArgs&, int64_t, hipStream_t);
template hipError_t launch_column_main<double>(Kind, const ColArgs&, int64_t, hipStream_t);
template hipError_t launch_column_main<float>(Kind, const ColArgs&, int64_t, hipStream_t);
template hipError_t launch_column_finalize<double>(Kind, const ColArgs&, int64_t, hipStream_t);
template hipError_t launch_column_finalize<float>(Kind, const ColArgs&, int64_t, hipStream_t);

}  // namespace pcg
