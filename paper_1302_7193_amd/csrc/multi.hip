// Multi-request kernels of the serving runtime (multi.h): thin wrappers that
// find a workgroup's request in the slot table and run the column kernel's
// body for it.
#include "kernels.h"
#include "multi.h"

namespace pcg {
namespace {

// Slot of workgroup t (the table's start[] ascending, start[0] = 0): a scalar
// walk over at most kMaxSlots entries.
__device__ __forceinline__ int find_slot(const MultiTable* tab, int64_t t)
{
    int s = 0;
    const int n = tab->nslots;
    while (s + 1 < n && tab->start[s + 1] <= t) ++s;
    return s;
}

template <MultiOp OP>
__global__ __launch_bounds__(kBlock) void k_multi(const MultiTable* __restrict__ tab)
{
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    const int s = find_slot(tab, t);
    const ColArgs& a = tab->args[s];
    const int64_t local = t - tab->start[s];
    if constexpr (OP == MultiOp::ApplyF32)
        fused_apply_dev<float, kServeM32, true, false, false, false>(a, local);
    else if constexpr (OP == MultiOp::PrecF32)
        fused_prec_dev<float, kServeM32, true, false, false, false>(a, local);
    else if constexpr (OP == MultiOp::ApplyF64)
        fused_apply_dev<double, kServeM64, true, false, false, false>(a, local);
    else if constexpr (OP == MultiOp::PrecF64)
        fused_prec_dev<double, kServeM64, true, false, false, false>(a, local);
    else if constexpr (OP == MultiOp::FixupF64)
        fixup_dev<double, kServeM64, true, false, false>(a, local);
    else if constexpr (OP == MultiOp::Residual64)
        residual64_dev<kServeM64, true, false, false, false>(a, local);
    else
        update64_dev<kServeM64, true, false, false>(a, local);
}

// One workgroup per slot: that request's finalize.
template <Kind K>
__global__ __launch_bounds__(kFinalThreads) void k_multi_finalize(const MultiTable* __restrict__ tab)
{
    finalize_dev<K>(tab->args[blockIdx.x], 0);
}

template <MultiOp OP>
hipError_t launch2(const MultiTable* tab, int64_t blocks, int nslots, hipStream_t s, Kind fin)
{
    hipLaunchKernelGGL((k_multi<OP>), dim3((unsigned)blocks), dim3(kBlock), 0, s, tab);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (fin) {
    case Kind::FusedApply:
        hipLaunchKernelGGL((k_multi_finalize<Kind::FusedApply>), dim3((unsigned)nslots),
                           dim3(kFinalThreads), 0, s, tab);
        break;
    case Kind::FusedPrec:
        hipLaunchKernelGGL((k_multi_finalize<Kind::FusedPrec>), dim3((unsigned)nslots),
                           dim3(kFinalThreads), 0, s, tab);
        break;
    case Kind::Fixup:
        hipLaunchKernelGGL((k_multi_finalize<Kind::Fixup>), dim3((unsigned)nslots),
                           dim3(kFinalThreads), 0, s, tab);
        break;
    case Kind::Residual64:
        hipLaunchKernelGGL((k_multi_finalize<Kind::Residual64>), dim3((unsigned)nslots),
                           dim3(kFinalThreads), 0, s, tab);
        break;
    default: return hipSuccess;   // no finalize
    }
    return hipGetLastError();
}

}  // namespace

hipError_t multi_launch(MultiOp op, const MultiTable* tab, int64_t blocks, int nslots,
                        hipStream_t s)
{
    if (blocks < 1 || nslots < 1 || nslots > kMaxSlots) return hipErrorInvalidValue;
    switch (op) {
    case MultiOp::ApplyF32: return launch2<MultiOp::ApplyF32>(tab, blocks, nslots, s, Kind::FusedApply);
    case MultiOp::PrecF32: return launch2<MultiOp::PrecF32>(tab, blocks, nslots, s, Kind::FusedPrec);
    case MultiOp::ApplyF64: return launch2<MultiOp::ApplyF64>(tab, blocks, nslots, s, Kind::FusedApply);
    case MultiOp::PrecF64: return launch2<MultiOp::PrecF64>(tab, blocks, nslots, s, Kind::FusedPrec);
    case MultiOp::FixupF64: return launch2<MultiOp::FixupF64>(tab, blocks, nslots, s, Kind::Fixup);
    case MultiOp::Residual64:
        return launch2<MultiOp::Residual64>(tab, blocks, nslots, s, Kind::Residual64);
    case MultiOp::Update64: return launch2<MultiOp::Update64>(tab, blocks, nslots, s, Kind::Apply);
    }
    return hipErrorInvalidValue;
}

}  // namespace pcg
