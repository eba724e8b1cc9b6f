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
#include <type_traits>

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

// y = A x from the CSR arrays, streamed through LDS (the CSR-stream scheme of
// Greathouse and Daga, SC 2014).  A workgroup takes kCsrRows consecutive
// rows; their entries are consecutive in the value and column arrays, so its
// lanes read them with 16-byte loads in one coalesced sweep (from the
// 16-byte boundary at or below the first entry), gather x for the entries of
// the rows, and write the products to LDS.  After a barrier lane t adds the
// products of row t in entry order and writes y.  Every load of the sweep is
// issued before any gather: a row has at most seven entries, so the sweep's
// length and the number of its steps per lane are bounded at compile time.
constexpr int kCsrRows = kBlock;
constexpr int kCsrMaxEntries = 7 * kCsrRows;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_csr_apply(int32_t n, const T* __restrict__ val,
                                                      const int32_t* __restrict__ col,
                                                      const int32_t* __restrict__ rowp,
                                                      const T* __restrict__ x, T* __restrict__ y)
{
    constexpr int V = 16 / sizeof(T);                        // entries per 16-byte load
    constexpr int kSteps = (kCsrMaxEntries + V - 1 + kBlock * V - 1) / (kBlock * V);
    using VT = std::conditional_t<sizeof(T) == 8, double2, float4>;
    using CT = std::conditional_t<sizeof(T) == 8, int2, int4>;
    __shared__ T prod[kCsrMaxEntries];
    __shared__ int32_t off[kCsrRows + 1];
    const int t = threadIdx.x;
    const int32_t r0 = (int32_t)blockIdx.x * kCsrRows;
    const int32_t rows = min(kCsrRows, n - r0);
    const int32_t e0 = rowp[r0], e1 = rowp[r0 + rows];
    if (t < rows) off[t] = rowp[r0 + t] - e0;
    if (t == 0) off[rows] = e1 - e0;
    // the sweep: [e0 rounded down to V, e1) in steps of kBlock * V entries;
    // the arrays' sections are padded to 256 bytes, so a 16-byte load that
    // starts below e1 stays inside its section
    const int32_t a0 = e0 & ~(V - 1);
    T v[kSteps][V];
    int32_t c[kSteps][V];
#pragma unroll
    for (int s = 0; s < kSteps; ++s) {
        const int32_t e = a0 + (s * kBlock + t) * V;
        if (e < e1) {
            const VT vv = *reinterpret_cast<const VT*>(val + e);
            const CT cv = *reinterpret_cast<const CT*>(col + e);
            if constexpr (V == 2) {
                v[s][0] = vv.x; v[s][1] = vv.y;
                c[s][0] = cv.x; c[s][1] = cv.y;
            } else {
                v[s][0] = vv.x; v[s][1] = vv.y; v[s][2] = vv.z; v[s][3] = vv.w;
                c[s][0] = cv.x; c[s][1] = cv.y; c[s][2] = cv.z; c[s][3] = cv.w;
            }
        }
    }
#pragma unroll
    for (int s = 0; s < kSteps; ++s) {
        const int32_t e = a0 + (s * kBlock + t) * V;
#pragma unroll
        for (int q = 0; q < V; ++q) {
            // entries outside the rows (before e0, at or after e1) are not
            // this workgroup's; their column slots may be padding
            if (e + q >= e0 && e + q < e1) prod[e + q - e0] = v[s][q] * x[c[s][q]];
        }
    }
    __syncthreads();
    if (t < rows) {
        T sum = T(0);
        for (int32_t e = off[t]; e < off[t + 1]; ++e) sum += prod[e];
        y[r0 + t] = sum;
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
    // n * 7 < 2^31 (checked when the problem is made): every row and entry
    // index fits in 32 bits
    const int32_t n = (int32_t)g.n;
    const dim3 grid((unsigned)((n + kCsrRows - 1) / kCsrRows)), block(kBlock);
    void* b = const_cast<void*>(buf);
    if (dtype == PCG_F64) {
        double* v; int32_t *c, *r;
        sections<double>(g, b, v, c, r);
        hipLaunchKernelGGL((k_csr_apply<double>), grid, block, 0, s, n, v, c, r,
                           static_cast<const double*>(x), static_cast<double*>(y));
    } else {
        float* v; int32_t *c, *r;
        sections<float>(g, b, v, c, r);
        hipLaunchKernelGGL((k_csr_apply<float>), grid, block, 0, s, n, v, c, r,
                           static_cast<const float*>(x), static_cast<float*>(y));
    }
    return hipGetLastError();
}

}  // namespace pcg
