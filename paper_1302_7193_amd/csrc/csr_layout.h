// Row offsets of the assembled-CSR comparator in closed form.  Rows follow
// the cell order (i*n_y + j)*n_z + k; a row holds the diagonal, its
// existing horizontal neighbours (two per periodic direction, one or two per
// Dirichlet direction) and its vertical neighbours (none across the bottom
// and top faces).  Host- and device-callable; compiled by g++ in the tests.
#pragma once

#include <cstdint>

#if defined(__HIPCC__)
#define PCG_HD __host__ __device__
#else
#define PCG_HD
#endif

namespace pcg {
namespace csr {

// Existing horizontal neighbours of index i (of n) in one direction.
PCG_HD inline int64_t nb_count(int64_t i, int64_t n, int per)
{
    if (per) return 2;
    return (i > 0) + (i < n - 1);
}

// Sum of nb_count over 0 .. i-1.
PCG_HD inline int64_t nb_prefix(int64_t i, int64_t n, int per)
{
    if (per) return 2 * i;
    if (i <= 0) return 0;
    return (i - 1) + (i < n - 1 ? i : n - 1);
}

// Entries in rows 0 .. k-1 of one column whose cells have hz horizontal
// neighbours: each row holds 1 + hz + (k' > 0) + (k' < n_z - 1) entries.
PCG_HD inline int64_t col_prefix(int64_t k, int64_t nz, int64_t hz)
{
    int64_t v = 0;
    if (k > 0) v += k - 1;
    v += k < nz - 1 ? k : nz - 1;
    return k * (1 + hz) + v;
}

PCG_HD inline int64_t row_offset(int64_t nx, int64_t ny, int64_t nz, int per_x, int per_y,
                                 int64_t i, int64_t j, int64_t k)
{
    const int64_t vert_col = 2 * (nz - 1);
    const int64_t ey_all = nb_prefix(ny, ny, per_y);
    int64_t off = i * ny * nz + nz * ny * nb_prefix(i, nx, per_x) + i * nz * ey_all +
                  i * ny * vert_col;
    off += j * nz * (1 + nb_count(i, nx, per_x)) + nz * nb_prefix(j, ny, per_y) + j * vert_col;
    const int64_t hz = nb_count(i, nx, per_x) + nb_count(j, ny, per_y);
    return off + col_prefix(k, nz, hz);
}

PCG_HD inline int64_t total_nnz(int64_t nx, int64_t ny, int64_t nz, int per_x, int per_y)
{
    return row_offset(nx, ny, nz, per_x, per_y, nx, 0, 0);
}

}  // namespace csr
}  // namespace pcg
