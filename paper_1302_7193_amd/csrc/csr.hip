// Matrix-explicit comparator (Sec. 6.2): the same operator assembled on the
// device into compressed sparse row storage, and a hand-written CSR product.
// Buffer layout: values (dtype, nnz), column indices (int32, nnz), row
// offsets (int32, n+1), each section 256-byte aligned.  Within a row the
// entries are ordered (i-1,j,k), (i,j-1,k), (i,j,k-1), (i,j,k), (i,j,k+1),
// (i,j+1,k), (i+1,j,k); periodic wrap-around neighbours take the same slots
// and neighbours across Dirichlet faces are absent.  Row offsets follow in
// closed form from the number of neighbours of each cell, so the assembly
// needs no scan.
#include <algorithm>

#include "csr_layout.h"
#include "device_common.h"

namespace pcg {
namespace {

__host__ __device__ inline int64_t row_offset(const Geom& g, int64_t i, int64_t j, int64_t k)
{
    return csr::row_offset(g.nx, g.ny, g.nz, g.per_x, g.per_y, i, j, k);
}

__host__ __device__ inline int64_t total_nnz(const Geom& g)
{
    return csr::total_nnz(g.nx, g.ny, g.nz, g.per_x, g.per_y);
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

template <typename T>
__global__ __launch_bounds__(kBlock) void k_csr_build(Geom g, const double* __restrict__ vert,
                                                      const double* __restrict__ hgeo, T* val,
                                                      int32_t* col, int32_t* rowp)
{
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r > g.n) return;
    if (r == g.n) { rowp[g.n] = (int32_t)total_nnz(g); return; }
    const int64_t c = r / g.nz;
    const int k = (int)(r - c * g.nz);
    const int64_t i = c / g.ny, j = c - i * g.ny;
    int cx = 0, cy = 0;
    int64_t im, ip, jm, jp;
    if (i > 0) im = c - g.ny; else if (g.per_x) im = c + (int64_t)(g.nx - 1) * g.ny; else { im = -1; ++cx; }
    if (i < g.nx - 1) ip = c + g.ny; else if (g.per_x) ip = c - (int64_t)(g.nx - 1) * g.ny; else { ip = -1; ++cx; }
    if (j > 0) jm = c - 1; else if (g.per_y) jm = c + (g.ny - 1); else { jm = -1; ++cy; }
    if (j < g.ny - 1) jp = c + 1; else if (g.per_y) jp = c - (g.ny - 1); else { jp = -1; ++cy; }
    // |T| and the face weights alpha_{T,T'}: uniform, or from the per-index
    // widths and reciprocal centre distances of a stretched grid
    double area = g.area, wxm = g.ax, wxp = g.ax, wym = g.ay, wyp = g.ay;
    double alpha_t = (2 + cx) * g.ax + (2 + cy) * g.ay;
    if (hgeo) {
        const double* hx = hgeo;
        const double* hy = hgeo + 3 * (int64_t)g.nx;
        area = hx[i] * hy[j];
        wxm = hy[j] * hx[g.nx + i];
        wxp = hy[j] * hx[2 * g.nx + i];
        wym = hx[i] * hy[g.ny + j];
        wyp = hx[i] * hy[2 * g.ny + j];
        alpha_t = (wxm + wxp) + (wym + wyp);
    }
    const double s = vert[k], b = vert[g.nzp + k], cc = vert[2 * g.nzp + k], d = vert[3 * g.nzp + k];
    int64_t e = row_offset(g, i, j, k);
    rowp[r] = (int32_t)e;
    auto put = [&](int64_t column, double v) {
        val[e] = T(v);
        col[e] = (int32_t)column;
        ++e;
    };
    if (im >= 0) put(im * g.nz + k, d * wxm);
    if (jm >= 0) put(jm * g.nz + k, d * wym);
    if (k > 0) put(r - 1, area * cc);
    put(r, area * s - alpha_t * d);
    if (k < g.nz - 1) put(r + 1, area * b);
    if (jp >= 0) put(jp * g.nz + k, d * wyp);
    if (ip >= 0) put(ip * g.nz + k, d * wxp);
}

// y = A x from the CSR arrays.  Eight lanes share a row (a row has at most
// seven entries): lane s of the group takes entry rowp[r] + s, so a
// wavefront's loads of values and column indices cover the consecutive
// entries of its eight rows in one coalesced sweep; the group adds its
// products with two quad permutes and one swizzle across the group's halves.
// Each wavefront takes kCsrGroups such row groups at a time, their loads
// issued together (three dependent loads per row: offsets, entries, x).
constexpr int kCsrLanes = 8;
constexpr int kCsrGroups = 4;

template <typename T>
__device__ __forceinline__ T group8_sum(T v)
{
    v += dpp_move<kQuadXor1>(v, T(0));
    v += dpp_move<kQuadXor2>(v, T(0));
    // xor 4: swizzle in bit mode (and 0x1f, or 0, xor 4) within each 32 lanes
    constexpr int kXor4 = 0x1f | (4 << 10);
    if constexpr (sizeof(T) == 8) {
        const int64_t b = __builtin_bit_cast(int64_t, v);
        const int lo = __builtin_amdgcn_ds_swizzle((int)b, kXor4);
        const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), kXor4);
        return v + __builtin_bit_cast(T, ((int64_t)hi << 32) | (int64_t)(uint32_t)lo);
    } else {
        return v + __builtin_bit_cast(T, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, v), kXor4));
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_csr_apply(int64_t n, const T* __restrict__ val,
                                                      const int32_t* __restrict__ col,
                                                      const int32_t* __restrict__ rowp,
                                                      const T* __restrict__ x, T* __restrict__ y)
{
    constexpr int kRowsPerWave = (kWave / kCsrLanes) * kCsrGroups;
    const int lane = threadIdx.x & (kWave - 1), slot = lane & (kCsrLanes - 1);
    const int64_t wave = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * (kBlock / kWave);
    for (int64_t r0 = wave * kRowsPerWave; r0 < n; r0 += nwaves * kRowsPerWave) {
        int64_t r[kCsrGroups];
        int32_t e[kCsrGroups], e1[kCsrGroups];
        T v[kCsrGroups], xv[kCsrGroups];
        int32_t c[kCsrGroups];
#pragma unroll
        for (int u = 0; u < kCsrGroups; ++u) {
            r[u] = r0 + u * (kWave / kCsrLanes) + lane / kCsrLanes;
            const int64_t rr = r[u] < n ? r[u] : n - 1;
            e[u] = rowp[rr] + slot;
            e1[u] = r[u] < n ? rowp[rr + 1] : 0;
        }
#pragma unroll
        for (int u = 0; u < kCsrGroups; ++u) {
            const bool in = e[u] < e1[u];
            const int32_t ee = in ? e[u] : 0;
            v[u] = in ? val[ee] : T(0);
            c[u] = in ? col[ee] : 0;
        }
#pragma unroll
        for (int u = 0; u < kCsrGroups; ++u) xv[u] = x[c[u]];
#pragma unroll
        for (int u = 0; u < kCsrGroups; ++u) {
            const T sum = group8_sum(v[u] * xv[u]);
            if (slot == 0 && r[u] < n) y[r[u]] = sum;
        }
    }
}

template <typename T>
void sections(const Geom& g, void* buf, T*& val, int32_t*& col, int32_t*& rowp)
{
    const int64_t nnz = total_nnz(g);
    char* p = static_cast<char*>(buf);
    val = reinterpret_cast<T*>(p);
    p += align256(sizeof(T) * (size_t)nnz);
    col = reinterpret_cast<int32_t*>(p);
    p += align256(sizeof(int32_t) * (size_t)nnz);
    rowp = reinterpret_cast<int32_t*>(p);
}

}  // namespace

size_t csr_bytes(const Geom& g, int dtype)
{
    const size_t nnz = (size_t)total_nnz(g);
    const size_t vs = dtype == PCG_F64 ? 8 : 4;
    return align256(vs * nnz) + align256(4 * nnz) + align256(4 * ((size_t)g.n + 1));
}

hipError_t csr_build(const Geom& g, const double* vert64, const double* hgeo, int dtype, void* buf,
                     hipStream_t s)
{
    const dim3 grid((unsigned)((g.n + 1 + kBlock - 1) / kBlock)), block(kBlock);
    if (dtype == PCG_F64) {
        double* v; int32_t *c, *r;
        sections<double>(g, buf, v, c, r);
        hipLaunchKernelGGL((k_csr_build<double>), grid, block, 0, s, g, vert64, hgeo, v, c, r);
    } else {
        float* v; int32_t *c, *r;
        sections<float>(g, buf, v, c, r);
        hipLaunchKernelGGL((k_csr_build<float>), grid, block, 0, s, g, vert64, hgeo, v, c, r);
    }
    return hipGetLastError();
}

hipError_t csr_apply(const Geom& g, int dtype, const void* buf, const void* x, void* y,
                     hipStream_t s)
{
    const int64_t rows_per_block = (int64_t)(kBlock / kCsrLanes) * kCsrGroups;
    const int64_t blocks = std::min<int64_t>((g.n + rows_per_block - 1) / rows_per_block, 1 << 20);
    const dim3 grid((unsigned)blocks), block(kBlock);
    void* b = const_cast<void*>(buf);
    if (dtype == PCG_F64) {
        double* v; int32_t *c, *r;
        sections<double>(g, b, v, c, r);
        hipLaunchKernelGGL((k_csr_apply<double>), grid, block, 0, s, g.n, v, c, r,
                           static_cast<const double*>(x), static_cast<double*>(y));
    } else {
        float* v; int32_t *c, *r;
        sections<float>(g, b, v, c, r);
        hipLaunchKernelGGL((k_csr_apply<float>), grid, block, 0, s, g.n, v, c, r,
                           static_cast<const float*>(x), static_cast<float*>(y));
    }
    return hipGetLastError();
}

}  // namespace pcg
