/*
 * CPU oracle for the line-preconditioned conjugate gradient solver of
 * Mueller, Guo, Scheichl and Shi, "Matrix-free GPU implementation of a
 * preconditioned conjugate gradient solver for anisotropic elliptic PDEs"
 * (arXiv 1302.7193).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product path
 * (the HIP library) never links, calls or reads anything from here, and this
 * file shares no code, header, table or constant generator with it.
 *
 * Everything is plain FP64 and deliberately unoptimised: the operator is
 * written out as an explicitly assembled CSR matrix built from face
 * transmissibilities of a cell-centred finite-volume scheme, the
 * preconditioner is that same assembled matrix with the couplings between
 * different vertical columns dropped, each column block is solved by
 * textbook tridiagonal Gaussian elimination, and the Krylov method is the
 * standard (not loop-fused) preconditioned conjugate gradient.
 *
 * Paper sections followed:
 *   - Sec. 3.1 (eqs. ColumnRepresentation, ModelEqnCubedSphere,
 *     DiagonalMatrix, TridiagonalMatrix): cell-integrated unknowns on a
 *     tensor-product grid; each horizontal cell T carries a vertical column
 *     of n_z unknowns; the column block A_T is tridiagonal and the coupling
 *     A_{T,T'} to a horizontal neighbour is diagonal.
 *   - Sec. 3.2 (eq. GlobalColumnReprConversion): ordering l = n_z*(i*n_y+j)+k.
 *   - Sec. 4.1: left-preconditioned CG, stopping on the unpreconditioned
 *     residual; the vertical-line preconditioner drops the horizontal
 *     off-diagonal blocks and inverts each tridiagonal block.
 *   - Sec. 4.2: tridiagonal solve per column (Thomas algorithm).
 *
 * Readings of the paper taken here (flat box instead of the cubed sphere):
 *   - domain [0, n_x*dx] x [0, n_y*dy] x [0, H]; vertical spacing graded
 *     geometrically with ratio q, finest cell at k = 0 (the ground);
 *   - operator -div(K grad u) + u with K = diag(K_h, K_h, K_v); the "+u"
 *     term integrated over the cell gives the cell volume on the diagonal;
 *   - Dirichlet faces use the half-cell distance (ghost value = -u);
 *     periodic faces wrap around; top and bottom are always Dirichlet.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- grid --- */

/* Vertical cell thicknesses dz[0..nz-1], summing to H.  Geometric grading
 * dz[k+1] = q*dz[k] with the smallest cell at the bottom (Sec. 3.1 asks for
 * smaller spacings near the ground; the ratio-q law replaces the paper's
 * quadratic law).  q == 1 gives the uniform grid H/nz. */
void orc_vertical_spacing(int nz, double H, double q, double *dz)
{
    if (q == 1.0) {
        for (int k = 0; k < nz; ++k) dz[k] = H / nz;
        return;
    }
    double first = H * (q - 1.0) / (pow(q, nz) - 1.0);
    for (int k = 0; k < nz; ++k) dz[k] = first * pow(q, k);
}

/* Vertical diffusion coefficient from the anisotropy ratio
 *   gamma^2 = (K_v / dzbar^2) / (K_h / dx^2),   dzbar = H / nz,
 * i.e. the strength ratio of the vertical and horizontal couplings measured
 * at the mean vertical spacing (Sec. 3, eq. Anisotropy, read for a flat
 * grid with diffusion tensor diag(K_h, K_h, K_v)). */
double orc_kv_from_ratio(double gamma2, double k_h, double dx, double H, int nz)
{
    double dzbar = H / nz;
    return gamma2 * k_h * dzbar * dzbar / (dx * dx);
}

/* ------------------------------------------------------------ assembly --- */

static long cell_index(int i, int j, int k, int ny, int nz)
{
    return ((long)i * ny + j) * (long)nz + k;
}

/* The entries of row c = (i,j,k) of A.  Writes up to 7 (column, value)
 * pairs, the diagonal first, and returns their number.
 *
 * Horizontal cell widths dxs[0..nx-1] and dys[0..ny-1] (a tensor-product
 * grid, uniform or stretched; Sec. 3.1 allows any horizontal geometry, only
 * |T| and the face weights alpha_{T,T'} change).  Cell volume
 * V = dxs[i]*dys[j]*dz[k]:
 *   A_cc += V                                  (zero-order term)
 *   for every face f of the cell, transmissibility
 *     t_f = diffusion coefficient * face area / distance between centres:
 *     interior or periodic neighbour n:  A_cc += t_f,  A_cn -= t_f
 *     Dirichlet face (ghost value -u):   A_cc += diffusion * area / (half cell)
 * The distance between the centres of horizontal neighbours is the mean of
 * their widths (across the periodic seam too).  A neighbour that appears
 * twice (periodic direction of length 1 or 2) is stored twice. */
static int build_row(int nx, int ny, int nz, const double *dxs, const double *dys,
                     const double *dz, double k_h, double k_v, int per_x, int per_y,
                     int i, int j, int k, int32_t *col, double *val)
{
    long c = cell_index(i, j, k, ny, nz);
    double dx = dxs[i], dy = dys[j];
    double diag = dx * dy * dz[k];
    int pos = 1;
    /* faces normal to x: area dy*dz[k] */
    for (int s = -1; s <= 1; s += 2) {
        int ii = i + s;
        if (ii < 0 || ii >= nx) {
            if (!per_x) { diag += k_h * dy * dz[k] / (0.5 * dx); continue; }
            ii = (ii + nx) % nx;
        }
        double t = k_h * dy * dz[k] / (0.5 * (dx + dxs[ii]));
        diag += t;
        col[pos] = (int32_t)cell_index(ii, j, k, ny, nz);
        val[pos++] = -t;
    }
    /* faces normal to y: area dx*dz[k] */
    for (int s = -1; s <= 1; s += 2) {
        int jj = j + s;
        if (jj < 0 || jj >= ny) {
            if (!per_y) { diag += k_h * dx * dz[k] / (0.5 * dy); continue; }
            jj = (jj + ny) % ny;
        }
        double t = k_h * dx * dz[k] / (0.5 * (dy + dys[jj]));
        diag += t;
        col[pos] = (int32_t)cell_index(i, jj, k, ny, nz);
        val[pos++] = -t;
    }
    /* faces normal to z: area dx*dy; bottom and top are Dirichlet */
    if (k > 0) {
        double t = k_v * dx * dy / (0.5 * (dz[k - 1] + dz[k]));
        diag += t;
        col[pos] = (int32_t)(c - 1);
        val[pos++] = -t;
    } else {
        diag += k_v * dx * dy / (0.5 * dz[k]);
    }
    if (k < nz - 1) {
        double t = k_v * dx * dy / (0.5 * (dz[k] + dz[k + 1]));
        diag += t;
        col[pos] = (int32_t)(c + 1);
        val[pos++] = -t;
    } else {
        diag += k_v * dx * dy / (0.5 * dz[k]);
    }
    col[0] = (int32_t)c;
    val[0] = diag;
    return pos;
}

/* Assemble A in CSR on a grid with horizontal widths dxs[nx], dys[ny].
 * row_ptr has n+1 entries; col/val have room for 7n.  Returns the number of
 * stored entries. */
long orc_assemble_geom(int nx, int ny, int nz, const double *dxs, const double *dys,
                       double H, double q, double k_h, double k_v, int per_x, int per_y,
                       int64_t *row_ptr, int32_t *col, double *val)
{
    double *dz = (double *)malloc(sizeof(double) * (size_t)nz);
    orc_vertical_spacing(nz, H, q, dz);
    long pos = 0;
    row_ptr[0] = 0;
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j)
            for (int k = 0; k < nz; ++k) {
                pos += build_row(nx, ny, nz, dxs, dys, dz, k_h, k_v, per_x, per_y,
                                 i, j, k, col + pos, val + pos);
                row_ptr[cell_index(i, j, k, ny, nz) + 1] = pos;
            }
    free(dz);
    return pos;
}

static double *constant_widths(int n, double w)
{
    double *a = (double *)malloc(sizeof(double) * (size_t)n);
    for (int i = 0; i < n; ++i) a[i] = w;
    return a;
}

/* Assemble A on the uniform grid of cell size dx * dy. */
long orc_assemble(int nx, int ny, int nz, double dx, double dy, double H, double q,
                  double k_h, double k_v, int per_x, int per_y,
                  int64_t *row_ptr, int32_t *col, double *val)
{
    double *dxs = constant_widths(nx, dx), *dys = constant_widths(ny, dy);
    long pos = orc_assemble_geom(nx, ny, nz, dxs, dys, H, q, k_h, k_v, per_x, per_y,
                                 row_ptr, col, val);
    free(dxs);
    free(dys);
    return pos;
}

/* y = A x for a CSR matrix. */
void orc_csr_matvec(long n, const int64_t *row_ptr, const int32_t *col,
                    const double *val, const double *x, double *y)
{
    for (long r = 0; r < n; ++r) {
        double s = 0.0;
        for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) s += val[e] * x[col[e]];
        y[r] = s;
    }
}

/* ------------------------------------------------------ preconditioner --- */

/* The line preconditioner M is A with every coupling between different
 * vertical columns removed (Sec. 4.1: drop the second term of eq.
 * ModelEqnCubedSphere).  Extract its tridiagonal blocks from the assembled
 * matrix: lo[l] multiplies x[l-1], di[l] multiplies x[l], up[l] multiplies
 * x[l+1], all restricted to the column that contains row l. */
void orc_line_blocks(long n, int nz, const int64_t *row_ptr, const int32_t *col,
                     const double *val, double *lo, double *di, double *up)
{
    for (long r = 0; r < n; ++r) {
        long column = r / nz;
        lo[r] = di[r] = up[r] = 0.0;
        for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
            long c = col[e];
            if (c / nz != column) continue; /* horizontal coupling: dropped */
            if (c == r) di[r] += val[e];
            else if (c == r - 1) lo[r] += val[e];
            else if (c == r + 1) up[r] += val[e];
        }
    }
}

/* z = M^{-1} r: one tridiagonal solve per column by Gaussian elimination
 * without pivoting (the Thomas algorithm, Sec. 4.2).  work holds 2*nz
 * doubles.  Each column block is strictly diagonally dominant, so no
 * pivoting is needed. */
void orc_line_solve(long n, int nz, const double *lo, const double *di,
                    const double *up, const double *r, double *z, double *work)
{
    double *cp = work;       /* modified super-diagonal */
    double *dp = work + nz;  /* modified right-hand side */
    for (long base = 0; base < n; base += nz) {
        const double *a = lo + base, *b = di + base, *c = up + base, *d = r + base;
        cp[0] = c[0] / b[0];
        dp[0] = d[0] / b[0];
        for (int k = 1; k < nz; ++k) {
            double m = b[k] - a[k] * cp[k - 1];
            cp[k] = c[k] / m;
            dp[k] = (d[k] - a[k] * dp[k - 1]) / m;
        }
        z[base + nz - 1] = dp[nz - 1];
        for (int k = nz - 2; k >= 0; --k) z[base + k] = dp[k] - cp[k] * z[base + k + 1];
    }
}

/* ------------------------------------------------------------------ PCG --- */

static double dot(long n, const double *a, const double *b)
{
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Standard preconditioned conjugate gradient (Sec. 4.1) on the assembled
 * matrix with the line preconditioner.  x holds x0 on entry and the
 * solution on exit.  Stops when ||r|| / ||r0|| < rtol or ||r|| < atol
 * (2-norm of the recursively updated unpreconditioned residual, as in the
 * exit test of Alg. InterleavedPCG), or after max_iter iterations.
 * An iteration is one product q = A p with its updates of x and r.
 *
 * out[0] = iterations, out[1] = recursive ||r||/||r0||, out[2] = ||r0||,
 * out[3] = true ||b - A x|| / ||r0||.
 * trace (optional, may be NULL) receives, for iterations 0..max_iter, the
 * vectors x_k, r_k, z_k, p_k (4n doubles per iteration); p_k is the search
 * direction used in iteration k+1.
 * Returns 0 on convergence, 1 if max_iter was reached, 2 on breakdown. */
int orc_pcg(long n, int nz, const int64_t *row_ptr, const int32_t *col, const double *val,
            const double *lo, const double *di, const double *up,
            const double *b, double *x, double rtol, double atol, int max_iter,
            double *out, double *trace)
{
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    double *work = (double *)malloc(sizeof(double) * 2 * (size_t)nz);
    int status = 1, it = 0;

    orc_csr_matvec(n, row_ptr, col, val, x, q);
    for (long i = 0; i < n; ++i) r[i] = b[i] - q[i];
    double r0 = sqrt(dot(n, r, r));
    double rn = r0;
    orc_line_solve(n, nz, lo, di, up, r, z, work);
    memcpy(p, z, sizeof(double) * (size_t)n);
    double rho = dot(n, r, z);
    if (trace) {
        memcpy(trace, x, sizeof(double) * (size_t)n);
        memcpy(trace + n, r, sizeof(double) * (size_t)n);
        memcpy(trace + 2 * n, z, sizeof(double) * (size_t)n);
        memcpy(trace + 3 * n, p, sizeof(double) * (size_t)n);
    }
    if (r0 == 0.0 || r0 < atol) {
        status = 0;
    } else {
        while (it < max_iter) {
            orc_csr_matvec(n, row_ptr, col, val, p, q);
            double pq = dot(n, p, q);
            if (!(pq > 0.0) || !isfinite(pq)) { status = 2; break; }
            double alpha = rho / pq;
            for (long i = 0; i < n; ++i) x[i] += alpha * p[i];
            for (long i = 0; i < n; ++i) r[i] -= alpha * q[i];
            ++it;
            rn = sqrt(dot(n, r, r));
            if (!isfinite(rn)) { status = 2; break; }
            int done = (rn / r0 < rtol) || (rn < atol);
            orc_line_solve(n, nz, lo, di, up, r, z, work);
            double rho_new = dot(n, r, z);
            if (!done && (!(rho_new > 0.0) || !isfinite(rho_new))) { status = 2; break; }
            double beta = rho_new / rho;
            rho = rho_new;
            for (long i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
            if (trace) {
                double *t = trace + (size_t)it * 4 * (size_t)n;
                memcpy(t, x, sizeof(double) * (size_t)n);
                memcpy(t + n, r, sizeof(double) * (size_t)n);
                memcpy(t + 2 * n, z, sizeof(double) * (size_t)n);
                memcpy(t + 3 * n, p, sizeof(double) * (size_t)n);
            }
            if (done) { status = 0; break; }
        }
    }
    orc_csr_matvec(n, row_ptr, col, val, x, q);
    for (long i = 0; i < n; ++i) q[i] = b[i] - q[i];
    out[0] = it;
    out[1] = r0 > 0.0 ? rn / r0 : 0.0;
    out[2] = r0;
    out[3] = r0 > 0.0 ? sqrt(dot(n, q, q)) / r0 : 0.0;
    free(r); free(z); free(p); free(q); free(work);
    return status;
}

/* True residual norm ||b - A x||_2 of any FP64 vector x. */
double orc_residual_norm(long n, const int64_t *row_ptr, const int32_t *col,
                         const double *val, const double *b, const double *x)
{
    double s = 0.0;
    for (long r = 0; r < n; ++r) {
        double ax = 0.0;
        for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) ax += val[e] * x[col[e]];
        double d = b[r] - ax;
        s += d * d;
    }
    return sqrt(s);
}

/* Row (i,j,k) of A x, for sampled checks on grids too large to assemble
 * (horizontal widths dxs[nx], dys[ny]). */
double orc_row_apply_geom(int nx, int ny, int nz, const double *dxs, const double *dys,
                          double H, double q, double k_h, double k_v, int per_x, int per_y,
                          int i, int j, int k, const double *x)
{
    int32_t col[7];
    double val[7];
    double *dz = (double *)malloc(sizeof(double) * (size_t)nz);
    orc_vertical_spacing(nz, H, q, dz);
    int cnt = build_row(nx, ny, nz, dxs, dys, dz, k_h, k_v, per_x, per_y, i, j, k, col, val);
    double s = 0.0;
    for (int e = 0; e < cnt; ++e) s += val[e] * x[col[e]];
    free(dz);
    return s;
}

/* The same on the uniform grid of cell size dx * dy. */
double orc_row_apply(int nx, int ny, int nz, double dx, double dy, double H, double q,
                     double k_h, double k_v, int per_x, int per_y,
                     int i, int j, int k, const double *x)
{
    double *dxs = constant_widths(nx, dx), *dys = constant_widths(ny, dy);
    double s = orc_row_apply_geom(nx, ny, nz, dxs, dys, H, q, k_h, k_v, per_x, per_y,
                                  i, j, k, x);
    free(dxs);
    free(dys);
    return s;
}
