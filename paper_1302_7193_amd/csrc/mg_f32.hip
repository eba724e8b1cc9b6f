// Multigrid kernels in FP32 (gfx950).
#include "mg.h"

namespace pcg {
template const void* mg_func<float>(Kind, const ColArgs&, int64_t);
}  // namespace pcg
