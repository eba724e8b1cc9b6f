// FP64 instances of the column-kernel launchers (kernels.h), and the launch
// helper shared by both precisions.
#include "kernels.h"

namespace pcg {

hipError_t issue(const KernelLaunch& k, hipStream_t s)
{
    void* args[] = {const_cast<ColArgs*>(&k.args)};
    return hipLaunchKernel(k.func, k.grid, k.block, args, 0, s);
}

template int column_launches<double>(Kind, const ColArgs&, int64_t, KernelLaunch*);
template hipError_t launch_column<double>(Kind, const ColArgs&, int64_t, hipStream_t);
template hipError_t launch_column_main<double>(Kind, const ColArgs&, int64_t, hipStream_t);
template hipError_t launch_column_finalize<double>(Kind, const ColArgs&, int64_t, hipStream_t);

}  // namespace pcg
