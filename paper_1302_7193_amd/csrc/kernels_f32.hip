// FP32 instances of the column-kernel launchers (kernels.h).
#include "kernels.h"

namespace pcg {

template int column_launches<float>(Kind, const ColArgs&, int64_t, KernelLaunch*);
template hipError_t launch_column<float>(Kind, const ColArgs&, int64_t, hipStream_t);
template hipError_t launch_column_main<float>(Kind, const ColArgs&, int64_t, hipStream_t);
template hipError_t launch_column_finalize<float>(Kind, const ColArgs&, int64_t, hipStream_t);

}  // namespace pcg
