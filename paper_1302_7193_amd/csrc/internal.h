// Internal declarations of libpcg: problem tables, device solver state,
// kernel argument blocks and the host-side launchers.  Everything here is
// private to the library; the public interface is include/pcg.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "pcg.h"

namespace pcg {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kBlock = 256;        // threads per workgroup of the column kernels
constexpr int kMaxNz = 1024;       // columns up to 64 lanes x 16 levels
constexpr int kClasses = 9;        // column classes: Dirichlet faces in x (0..2) x in y (0..2)
constexpr int kRedSlots = 2;       // doubles per workgroup in the partial-sum buffer
// Vectors of the fused iteration larger than this are streamed with the
// nontemporal hint: they cannot stay in the caches (32 MB of L2, 256 MB of
// Infinity Cache) from one kernel to the next.  Only when a lane moves one
// 16-byte chunk per vector, so that every store instruction of a wavefront
// covers whole cache lines: with two or more chunks per lane each
// instruction writes every other chunk, and nontemporal stores of such
// partial lines raised the measured write traffic by a tenth.
constexpr int64_t kStreamBytes = int64_t(64) << 20;
// Kernel B stores z with the default cache policy, not the nontemporal
// hint, when the z vectors of all right-hand sides take at most this many
// bytes: kernel A reads z right after (with its neighbour columns), and the
// part that stays in the 256 MB Infinity Cache is not read from HBM again.
// Measured: 268 MB of FP64 z (512 x 512 x 128) made kernels A and B 8 and 7 %
// faster; 512 MB of FP32 z (1024 x 1024 x 128) made the solve 3 % slower.
constexpr int64_t kCacheZBytes = int64_t(384) << 20;
constexpr int64_t kMaxBlocks = 65536;   // largest workgroup cap per right-hand side
constexpr int64_t kDefaultCap = 16384;  // default workgroup cap per right-hand side
// Fixed device scratch of the allocation-free solve (per device, for the
// life of the process): an FP64 solve of up to about 2 million unknowns.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr double kMgOmega = 0.8;   // multigrid: damping of the line-Jacobi smoother
constexpr int kMgMinCells = 4;     // coarsen while both halves keep >= 4 cells
constexpr int kMgCoarseSweeps = 4; // smoothing sweeps from zero on the coarsest level

// Solver flags kept in device memory.
enum : int32_t {
    kRunning = 0,
    kConverged = 1,   // exit test met; x still lacks alpha*p
    kMaxIter = 2,     // iteration limit; x still lacks alpha*p
    kBreakdown = 3,   // non-positive or non-finite curvature / residual
};

// Device-resident scalars of one Krylov solve (all FP64, Alg. InterleavedPCG:
// alpha, beta, kappa_old, sigma, ||r||, ||r0||).  One per right-hand side.
struct alignas(128) SolverState {
    double alpha;
    double beta;
    double kappa_old;
    double rnorm;
    double r0norm;
    double sigma;
    double rtol;
    double atol;
    double aux;        // free slot (true residual norm, refinement scale)
    int32_t flag;
    int32_t iter;      // completed iterations (applications of A to p)
    int32_t max_iter;
    int32_t fixed;     // exit correction x += alpha*p applied
    uint32_t ticket;   // last-workgroup counter of the current reduction
    int32_t zero_start;// x0 = 0: the first kernel B reads b, x is not read
    int32_t pad[2];
};

// Per-column geometry of the flat tensor-product grid.  The paper's
// |T| (cell area) and alpha_{T,T'} (edge length / centre distance) are
// rebuilt from these in every kernel, once per column (Sec. 4.2).
struct Geom {
    int32_t nx, ny, nz, nzp;   // nzp: n_z padded to a multiple of 4
    int32_t per_x, per_y;
    int64_t nh;                // columns
    int64_t n;                 // cells
    double area;               // |T| = dx*dy
    double ax, ay;             // alpha_{T,T'} for x and y neighbours
};

// Column tables in device memory, for one precision T:
//   vert[9][nzp]     s_k = a_k - b_k - c_k, b_k, c_k, d_k (eq. TridiagonalMatrix),
//                    then, for factorising stretched-grid column blocks in the
//                    kernel with every quantity scaled by s_k (well inside the
//                    FP32 range however fine the vertical grid):
//                    e_k = -d_k / s_k, pi_k = c_k b_{k-1} / (s_k s_{k-1}),
//                    cs_k = c_k / s_{k-1}, bs_k = b_k / s_k, is_k = 1 / s_k
//                    (pi_0 = cs_0 = 0, bs_{n_z-1} = 0)
//   lu[9][3][nzp]    per column class: l_k, 1/D_k, phi_k of the LU factors of
//                    the column block A_T (zero beyond n_z)
template <typename T>
struct Tables {
    const T* vert;
    const T* lu;
};

// Launch shape of the column kernels: L lanes per column, each lane owns M
// consecutive levels (L*M >= n_z); 64/L columns per wave; 4 waves per
// workgroup.
struct Shape {
    int L = 16;
    int M = 4;
    int cols_per_block() const { return (kWave / L) * (kBlock / kWave); }
};

// Tunable launch parameters of one precision (see pcg_tuning).
struct Tuning {
    Shape shape;
    int64_t block_cap = kDefaultCap;   // workgroups per right-hand side
    int red_mode = 1;           // reduction mode (ColArgs::red_mode)
    Shape shape_b;              // the same two for the line-solve kernels
    int64_t block_cap_b = kDefaultCap;   // (kernel B, the preconditioner alone)
};

// ---------------------------------------------------------------- kernels --

enum class Kind : int {
    Apply,        // y = A x
    Precond,      // z = M^{-1} r
    InitFull,     // r = b - A x
    InitZero,     // r = b, x = 0, p = q = 0 (unfused start)
    FusedPrec,    // kernel B: r -= alpha q; z = M^{-1} r; R, kappa; exit test; beta
    FusedApply,   // kernel A: x += alpha p; p = z + beta p; q = A z + beta q; sigma; alpha
    Fixup,        // x += alpha p once, after the exit test fired
    Residual64,   // FP64 r = b - A x, ||r||; FP32 copy r * scale  (refinement)
    Update64,     // FP64 x += (u32 + alpha p32) / scale           (refinement)
    TrueResidual, // FP64 ||b - A x||
    FusedPrecFirst,  // kernel B's first launch in a solve (alpha = 0, q unset)
    FusedApplyFirst, // kernel A's first launch in a solve (p = z, q = A z)
    // tensor-product multigrid preconditioner (mg.hip), on one level each:
    MgPre,        // z = omega M^{-1} r                      (pre-smoothing from zero)
    MgPreFused,   // the same, first: r -= alpha q, as kernel B does
    MgRestrict,   // coarse r = P^T (r - A z)                 (tiles of the coarse level)
    MgPost,       // z += P z_c; z += omega M^{-1}(r - A z)   (post-smoothing)
    MgPostFinal,  // the same, then R, kappa; exit test; beta  (ends kernel B's work)
    MgSmooth,     // z += omega M^{-1}(r - A z)               (coarsest level)
    MgSmoothFinal,// the same, then R, kappa; exit test; beta  (single-level hierarchy)
    // symmetric red-black block Gauss-Seidel (rbgs.hip):
    RbFirst,      // red columns: z = D^{-1} r
    RbFirstFused, // the same, first: r -= alpha q on every column, as kernel B does
    RbBlack,      // black columns: z = D^{-1}(r - A_BR z)
    RbRed,        // red columns:   z = D^{-1}(r - A_RB z)
    RbRedFinal,   // the same, then R, kappa over all columns; exit test; beta
};

// One argument block serves every column kernel; unused pointers are null.
// `batch` right-hand sides are stacked with stride n; block b of the grid
// covers right-hand side b / blocks_per_rhs.
struct ColArgs {
    Geom g;
    int L;
    int64_t blocks_per_rhs;
    int L_b;                // launch shape of the line-solve kernels (FusedPrec,
    int64_t bpr_b;          // Precond): column_launches moves it into L and
                            // blocks_per_rhs for those kinds
    const void* vert;   // Tables<T>::vert
    const void* lu;     // Tables<T>::lu
    const void* in0;    // x (Apply/Init), r (Precond), ...
    const void* in1;    // b
    void* io0;          // x / u
    void* io1;          // r
    void* io2;          // z
    void* io3;          // p
    void* io4;          // q
    void* out32;        // FP32 vector of the refinement kernels
    SolverState* st;    // per right-hand side
    double* part;       // [batch][blocks_per_rhs][values reduced (1 or 2)]
    int red_mode;       // 0: last workgroup finishes reductions; 1: finalize launch
    int x0_zero;        // x is zero (not read): refinement kernels, and kernel B's first
                        // launch, which then takes r from b
    const double* hgeo; // stretched grids: per-index widths and face weights
                        // [w_x m_x p_x](n_x) [w_y m_y p_y](n_y); null when uniform
    // multigrid kernels: the other level of an intergrid transfer (the fine
    // level for MgRestrict, the coarse one for MgPost*), its geometry table,
    // and the smoother's damping
    Geom g2;
    const double* hgeo2;
    double omega;
    // fused iteration with the line preconditioner: kernel A's first launch
    // does not store p = z (z stays in io2 and serves as that p); from the
    // first iteration on kernel B writes z into io3 and kernel A keeps p in
    // io2 (in place), so the two vectors swap roles.  On a zero start kernel
    // B's first launch does not copy b into r: its second reads b (in1)
    int zswap;
    // mixed-precision update: the states of the inner solves whose pending
    // exit correction (u += alpha p) it folds in; null elsewhere
    const SolverState* st_in;
    // kernel B stores z without the nontemporal hint (kCacheZBytes)
    int cache_z;
};

// Multigrid kernels (mg.hip): kernel for a Kind in MgPre..MgSmoothFinal, or
// null; block Gauss-Seidel kernels (rbgs.hip): Kind >= RbFirst.
template <typename T>
const void* mg_func(Kind kind, const ColArgs& a, int64_t batch);
template <typename T>
const void* rb_func(Kind kind, const ColArgs& a, int64_t batch);

// Host launchers (kernels.h): T = double or float.  column_launches
// returns the kernel (and, for mode-1 reductions, its finalize kernel) with
// launch dimensions, for direct launches or graph nodes; launch_column
// issues both; launch_column_main / launch_column_finalize issue them
// separately.
struct KernelLaunch {
    const void* func;
    dim3 grid;
    dim3 block;
    ColArgs args;       // the argument block of this launch
};
template <typename T>
int column_launches(Kind kind, const ColArgs& a, int64_t batch, KernelLaunch out[2]);
hipError_t issue(const KernelLaunch& k, hipStream_t s);
template <typename T>
hipError_t launch_column(Kind kind, const ColArgs& a, int64_t batch, hipStream_t s);
template <typename T>
hipError_t launch_column_main(Kind kind, const ColArgs& a, int64_t batch, hipStream_t s);
template <typename T>
hipError_t launch_column_finalize(Kind kind, const ColArgs& a, int64_t batch, hipStream_t s);

// Unfused BLAS-1 style kernels with device-resident scalars (blas.hip).
enum class Blas : int {
    DotPQ,        // sigma = <p,q>; alpha = rho / sigma
    DotRZ,        // rho' = <r,z>; beta = rho'/rho; rho = rho'
    Nrm2R,        // ||r||; exit test; iteration count
    AxpyXP,       // x += alpha p
    AxpyRQ,       // r -= alpha q
    ScalP,        // p = beta p
    AxpyPZ,       // p += z
    CopyZP,       // p = z (start)
    InitDot,      // rho = <r,z>, ||r0|| (start)
};

struct BlasArgs {
    int64_t n;
    int64_t blocks;
    const double* x;
    const double* y;
    double* w0;
    double* w1;
    SolverState* st;
    double* part;
    int red_mode;       // as ColArgs::red_mode
};
hipError_t launch_blas(Blas op, const BlasArgs& a, hipStream_t s);

// CSR comparator (csr.hip).
size_t csr_bytes(const Geom& g, int dtype);
hipError_t csr_build(const Geom& g, const double* vert64, const double* hgeo, int dtype, void* buf,
                     hipStream_t s);
hipError_t csr_apply(const Geom& g, int dtype, const void* buf, const void* x, void* y,
                     hipStream_t s);

// Shape selection and the number of workgroups for a column kernel.
Shape default_shape(int nz, int dtype);
int64_t column_blocks(const Geom& g, const Shape& sh);
bool shape_supported(int nz, const Shape& sh);

// Error reporting (abi.cpp).
void set_error(const std::string& msg);

}  // namespace pcg
