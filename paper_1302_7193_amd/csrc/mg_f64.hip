// Multigrid kernels in FP64 (gfx950).
#include "mg.h"

namespace pcg {
template const void* mg_func<double>(Kind, const ColArgs&, int64_t);
}  // namespace pcg
