// Unfused comparator: the standard PCG iteration of Sec. 4.1 as separate
// sweeps over memory -- three axpy, one scal, two dot and one nrm2 per
// iteration (Tab. BLASoperations) beside the operator and preconditioner
// kernels.  FP64.  Scalars stay in device memory: the scalar step each
// reduction enables runs on the device (in the last workgroup, or in a
// one-workgroup finalize launch), so no host round trip is needed between
// kernels.
#include "device_common.h"

namespace pcg {
namespace {

// Scalar step that a reduction enables (standard PCG, Sec. 4.1).
template <Blas OP>
__device__ inline void blas_finish(SolverState* s, const double (&tot)[2])
{
    if (OP == Blas::DotPQ) {          // alpha = rho / <p, Ap>
        if (!(tot[0] > 0.0) || !isfinite(tot[0])) { s->flag = kBreakdown; return; }
        s->sigma = tot[0];
        s->alpha = s->kappa_old / tot[0];
    } else if (OP == Blas::Nrm2R) {   // exit test on the updated residual
        const double rn = sqrt(tot[0]);
        s->rnorm = rn;
        s->iter += 1;
        if (!isfinite(rn)) s->flag = kBreakdown;
        else if (rn / s->r0norm < s->rtol || rn < s->atol) s->flag = kConverged;
        else if (s->iter >= s->max_iter) s->flag = kMaxIter;
    } else if (OP == Blas::DotRZ) {   // beta = rho' / rho
        if (!(tot[0] > 0.0) || !isfinite(tot[0])) { s->flag = kBreakdown; return; }
        s->beta = tot[0] / s->kappa_old;
        s->kappa_old = tot[0];
    } else if (OP == Blas::InitDot) { // start: rho = <r,z>, ||r0||
        const double rn = sqrt(tot[1]);
        s->r0norm = s->rnorm = rn;
        s->kappa_old = tot[0];
        if (!isfinite(rn) || !isfinite(tot[0])) s->flag = kBreakdown;
        else if (rn == 0.0 || rn < s->atol) s->flag = kConverged;
        else if (!(tot[0] > 0.0)) s->flag = kBreakdown;
    }
}

template <Blas OP>
__global__ __launch_bounds__(kBlock) void k_blas(BlasArgs a)
{
    SolverState* s = a.st;
    if (s->flag != kRunning) return;
    const int64_t nb = gridDim.x;
    const int64_t blk = xcd_remap(blockIdx.x, nb);
    const int64_t n2 = a.n >> 1;
    const int64_t b0 = blk * n2 / nb, b1 = (blk + 1) * n2 / nb;
    const double alpha = s->alpha, beta = s->beta;
    const double2* x2 = reinterpret_cast<const double2*>(a.x);
    const double2* y2 = reinterpret_cast<const double2*>(a.y);
    double2* w2 = reinterpret_cast<double2*>(a.w0);
    double acc[2] = {0.0, 0.0};
    auto body = [&](double x0, double y0, double& w) {
        switch (OP) {
        case Blas::DotPQ:
        case Blas::DotRZ: acc[0] += x0 * y0; break;
        case Blas::InitDot: acc[0] += x0 * y0; acc[1] += x0 * x0; break;
        case Blas::Nrm2R: acc[0] += x0 * x0; break;
        case Blas::AxpyXP: w += alpha * x0; break;
        case Blas::AxpyRQ: w -= alpha * x0; break;
        case Blas::ScalP: w *= beta; break;
        case Blas::AxpyPZ: w += x0; break;
        case Blas::CopyZP: w = x0; break;
        }
    };
    constexpr bool reads_y = OP == Blas::DotPQ || OP == Blas::DotRZ || OP == Blas::InitDot;
    constexpr bool reads_x = OP != Blas::ScalP;
    constexpr bool rw_w = OP == Blas::AxpyXP || OP == Blas::AxpyRQ || OP == Blas::ScalP ||
                          OP == Blas::AxpyPZ;
    constexpr bool wr_w = rw_w || OP == Blas::CopyZP;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += kBlock) {
        const double2 xv = reads_x ? x2[i] : double2{0.0, 0.0};
        const double2 yv = reads_y ? y2[i] : double2{0.0, 0.0};
        double2 wv = rw_w ? w2[i] : double2{0.0, 0.0};
        body(xv.x, yv.x, wv.x);
        body(xv.y, yv.y, wv.y);
        if (wr_w) w2[i] = wv;
    }
    if ((a.n & 1) && blk == nb - 1 && threadIdx.x == 0) {   // odd tail element
        const int64_t i = a.n - 1;
        double w = rw_w ? a.w0[i] : 0.0;
        body(reads_x ? a.x[i] : 0.0, reads_y ? a.y[i] : 0.0, w);
        if (wr_w) a.w0[i] = w;
    }
    constexpr bool reduces = OP == Blas::DotPQ || OP == Blas::DotRZ || OP == Blas::InitDot ||
                             OP == Blas::Nrm2R;
    if constexpr (reduces) {
        double tot[2];
        if (publish<2>(acc, a.part, blk, nb, &s->ticket, a.red_mode, tot) && threadIdx.x == 0)
            blas_finish<OP>(s, tot);
    }
}

// Mode-1 reductions of the BLAS-1 kernels (one workgroup).
template <Blas OP>
__global__ __launch_bounds__(kFinalThreads) void k_blas_finalize(BlasArgs a)
{
    SolverState* s = a.st;
    if (s->flag != kRunning) return;
    double tot[2];
    sum_partials<2, false, kFinalThreads>(a.part, a.blocks, tot);
    if (threadIdx.x == 0) blas_finish<OP>(s, tot);
}

}  // namespace

hipError_t launch_blas(Blas op, const BlasArgs& a, hipStream_t s)
{
    const dim3 grid((unsigned)a.blocks), block(kBlock);
    const bool fin = a.red_mode != 0 && (op == Blas::DotPQ || op == Blas::DotRZ ||
                                         op == Blas::Nrm2R || op == Blas::InitDot);
    switch (op) {
#define PCG_BLAS_CASE(X)                                                                \
    case Blas::X:                                                                       \
        hipLaunchKernelGGL((k_blas<Blas::X>), grid, block, 0, s, a);                    \
        if (fin) hipLaunchKernelGGL((k_blas_finalize<Blas::X>), dim3(1), dim3(kFinalThreads), 0, s, a); \
        break;
        PCG_BLAS_CASE(DotPQ)
        PCG_BLAS_CASE(DotRZ)
        PCG_BLAS_CASE(Nrm2R)
        PCG_BLAS_CASE(AxpyXP)
        PCG_BLAS_CASE(AxpyRQ)
        PCG_BLAS_CASE(ScalP)
        PCG_BLAS_CASE(AxpyPZ)
        PCG_BLAS_CASE(CopyZP)
        PCG_BLAS_CASE(InitDot)
#undef PCG_BLAS_CASE
    }
    return hipGetLastError();
}

}  // namespace pcg
