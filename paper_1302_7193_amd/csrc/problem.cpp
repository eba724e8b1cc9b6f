// Problem set-up: descriptor validation, the vertical coefficient vectors
// a, b, c, d of the column blocks (Sec. 3.1, eq. TridiagonalMatrix; Sec. 4.2:
// only O(n_z) numbers describe the vertical discretisation), and the LU
// factors of the column block of every column class.
#include <cmath>
#include <cstring>
#include <new>
#include <sstream>

#include "problem.h"

namespace pcg {

namespace {

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Vertical cell thicknesses: geometric grading with ratio q, finest at the
// bottom, summing to the height.
std::vector<double> thicknesses(int nz, double height, double q)
{
    std::vector<double> dz(nz);
    if (q == 1.0) {
        for (int k = 0; k < nz; ++k) dz[k] = height / nz;
    } else {
        const double h0 = height * (q - 1.0) / (std::pow(q, nz) - 1.0);
        double h = h0;
        for (int k = 0; k < nz; ++k) {
            dz[k] = h;
            h *= q;
        }
    }
    return dz;
}

}  // namespace

std::string validate(const pcg_problem_desc& d)
{
    std::ostringstream m;
    if (d.nx < 1 || d.ny < 1 || d.nz < 1) m << "grid sizes must be >= 1";
    else if (d.nz > kMaxNz) m << "nz = " << d.nz << " exceeds " << kMaxNz;
    else if ((int64_t)d.nx * d.ny * d.nz * 7 >= (int64_t)1 << 31)
        m << "n_x*n_y*n_z*7 must stay below 2^31 (int32 indices of the CSR comparator)";
    else if (!finite_pos(d.dx) || !finite_pos(d.dy) || !finite_pos(d.height))
        m << "dx, dy and height must be positive and finite";
    else if (!finite_pos(d.grading)) m << "grading must be positive and finite";
    else if (!(std::isfinite(d.k_h) && d.k_h >= 0.0)) m << "k_h must be finite and >= 0";
    else if (!finite_pos(d.k_v)) m << "k_v must be positive and finite";
    else if ((d.bc_x != PCG_BC_DIRICHLET && d.bc_x != PCG_BC_PERIODIC) ||
             (d.bc_y != PCG_BC_DIRICHLET && d.bc_y != PCG_BC_PERIODIC))
        m << "bc_x/bc_y must be PCG_BC_DIRICHLET or PCG_BC_PERIODIC";
    else if ((d.bc_x == PCG_BC_PERIODIC && d.nx < 3) || (d.bc_y == PCG_BC_PERIODIC && d.ny < 3))
        m << "periodic directions need at least 3 cells";
    return m.str();
}

// Tables for the column kernels.
//   a_k = dz_k                   zero-order term per unit area
//   d_k = -K_h dz_k              horizontal coupling per unit alpha_{T,T'}
//   b_k = -K_v / h_{k+1/2}       vertical coupling to level k+1 per unit area
//   c_k = -K_v / h_{k-1/2}       vertical coupling to level k-1 per unit area
// h_{k+1/2} is the distance between the centres of levels k and k+1, and
// half a cell at the bottom and top faces (Dirichlet), where b_{n_z-1} and
// c_0 carry the boundary coupling that only enters the diagonal.  The column
// block is then |T| diag(a) - alpha_T diag(d) + |T| tridiag(-(b+c), b, c).
void build_tables(const pcg_problem_desc& d, Geom& g, std::vector<double>& vert,
                  std::vector<double>& lu)
{
    const int nz = d.nz;
    g.nx = d.nx;
    g.ny = d.ny;
    g.nz = nz;
    g.nzp = (nz + 3) & ~3;
    g.per_x = d.bc_x == PCG_BC_PERIODIC;
    g.per_y = d.bc_y == PCG_BC_PERIODIC;
    g.nh = (int64_t)d.nx * d.ny;
    g.n = g.nh * nz;
    g.area = d.dx * d.dy;
    g.ax = d.dy / d.dx;   // edge length / centre distance across an x face
    g.ay = d.dx / d.dy;

    const std::vector<double> dz = thicknesses(nz, d.height, d.grading);
    const int nzp = g.nzp;
    vert.assign(9 * (size_t)nzp, 0.0);
    std::vector<double> b(nz), c(nz);
    for (int k = 0; k < nz; ++k) {
        const double a = dz[k];
        const double up = k < nz - 1 ? 0.5 * (dz[k] + dz[k + 1]) : 0.5 * dz[k];
        const double dn = k > 0 ? 0.5 * (dz[k - 1] + dz[k]) : 0.5 * dz[k];
        b[k] = -d.k_v / up;
        c[k] = -d.k_v / dn;
        vert[0 * nzp + k] = a - b[k] - c[k];
        vert[1 * nzp + k] = b[k];
        vert[2 * nzp + k] = c[k];
        vert[3 * nzp + k] = -d.k_h * dz[k];
    }
    for (int k = 0; k < nz; ++k) {
        const double sk = vert[k];
        vert[4 * nzp + k] = -vert[3 * nzp + k] / sk;
        vert[5 * nzp + k] = k > 0 ? (c[k] / sk) * (b[k - 1] / vert[k - 1]) : 0.0;
        vert[6 * nzp + k] = k > 0 ? c[k] / vert[k - 1] : 0.0;
        vert[7 * nzp + k] = k < nz - 1 ? b[k] / sk : 0.0;
        vert[8 * nzp + k] = 1.0 / sk;
    }

    // LU factors (no pivoting: every column block is strictly diagonally
    // dominant) for each class of column: cx, cy = number of Dirichlet side
    // faces in x and y, each counted twice in alpha_T (half-cell distance).
    lu.assign((size_t)kClasses * 3 * nzp, 0.0);
    for (int cls = 0; cls < kClasses; ++cls) {
        const int cx = cls / 3, cy = cls % 3;
        const double alpha_t = (2 + cx) * g.ax + (2 + cy) * g.ay;
        double* lf = &lu[((size_t)cls * 3 + 0) * nzp];
        double* inv_d = &lu[((size_t)cls * 3 + 1) * nzp];
        double* phi = &lu[((size_t)cls * 3 + 2) * nzp];
        double dprev = 0.0;
        for (int k = 0; k < nz; ++k) {
            const double diag = g.area * vert[k] - alpha_t * vert[3 * nzp + k];
            const double sub = k > 0 ? g.area * c[k] : 0.0;
            const double sup_prev = k > 0 ? g.area * b[k - 1] : 0.0;
            const double l = k > 0 ? sub / dprev : 0.0;
            const double dk = diag - l * sup_prev;
            lf[k] = l;
            inv_d[k] = 1.0 / dk;
            phi[k] = k < nz - 1 ? g.area * b[k] / dk : 0.0;
            dprev = dk;
        }
    }
}

// Stretched horizontal grids: per index i of a direction with widths w, the
// width w_i and the reciprocal centre distances to the lower and upper
// neighbour, m_i and p_i (half a width at a Dirichlet wall, so the face
// weight alpha_{T,T'} = edge length * m_i counts that face twice; across a
// periodic seam the distance joins the first and last cells).  Layout
// [w_x m_x p_x](n_x) [w_y m_y p_y](n_y).
std::string stretched_geometry(const pcg_problem_desc& d, const double* xw, const double* yw,
                               std::vector<double>& hgeo)
{
    for (int i = 0; i < d.nx; ++i)
        if (!finite_pos(xw[i])) return "x widths must be positive and finite";
    for (int j = 0; j < d.ny; ++j)
        if (!finite_pos(yw[j])) return "y widths must be positive and finite";
    hgeo.assign(3 * (size_t)d.nx + 3 * (size_t)d.ny, 0.0);
    auto fill = [](const double* w, int n, bool periodic, double* out) {
        for (int i = 0; i < n; ++i) {
            out[i] = w[i];
            const double lo = i > 0 ? 0.5 * (w[i - 1] + w[i])
                                    : (periodic ? 0.5 * (w[n - 1] + w[0]) : 0.5 * w[0]);
            const double hi = i < n - 1 ? 0.5 * (w[i] + w[i + 1])
                                        : (periodic ? 0.5 * (w[n - 1] + w[0]) : 0.5 * w[n - 1]);
            out[n + i] = 1.0 / lo;
            out[2 * n + i] = 1.0 / hi;
        }
    };
    fill(xw, d.nx, d.bc_x == PCG_BC_PERIODIC, hgeo.data());
    fill(yw, d.ny, d.bc_y == PCG_BC_PERIODIC, hgeo.data() + 3 * (size_t)d.nx);
    return "";
}

Shape default_shape(int nz, int dtype)
{
    Shape s;
    const int m_target = dtype == PCG_F64 ? 4 : 8;   // 32 bytes per lane per vector
    int L = 1;
    while (L * m_target < nz) L <<= 1;
    if (L > kWave) L = kWave;
    s.L = L;
    s.M = 1;
    while (s.M * L < nz) s.M <<= 1;
    return s;
}

bool shape_supported(int nz, const Shape& sh)
{
    if (sh.L < 1 || sh.L > kWave || (sh.L & (sh.L - 1))) return false;
    int M = 1;
    while (M * sh.L < nz) M <<= 1;
    return M <= 16;
}

int64_t column_blocks(const Geom& g, const Shape& sh)
{
    const int64_t cols = (int64_t)sh.cols_per_block();
    return (g.nh + cols - 1) / cols;
}

}  // namespace pcg
