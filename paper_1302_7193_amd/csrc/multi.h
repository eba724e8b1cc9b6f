// Multi-request launches of the serving runtime (continuous batching): one
// launch of a column kernel advances every request of a slot table, each
// request with its own grid, tables, vectors, solver state and partial sums.
// Workgroup t of such a launch belongs to the slot s with start[s] <= t <
// start[s + 1] and plays workgroup t - start[s] of that request's own
// launch, so a request's arithmetic and summation order are those of a
// launch of its own with the same launch shape.
#pragma once

#include "internal.h"

namespace pcg {

constexpr int kMaxSlots = 64;   // requests in one multi-request launch

struct MultiTable {
    int32_t nslots;
    int32_t pad;
    int64_t start[kMaxSlots + 1];   // first workgroup of each slot; start[nslots] = grid
    ColArgs args[kMaxSlots];
};

// The kernels a multi-request launch can run, all in the served launch
// shape (FP32 inner kernels with 4 levels per lane, FP64 refinement kernels
// with 2, lanes per column L = n_z / levels, vector path).
enum class MultiOp : int {
    ApplyF32,     // kernel A (FP32), with its finalize launch
    PrecF32,      // kernel B (FP32), with its finalize launch
    ApplyF64,     // kernel A (FP64)
    PrecF64,      // kernel B (FP64)
    FixupF64,     // exit correction (FP64), with its finalize launch
    Residual64,   // refinement residual, with its finalize launch
    Update64,     // refinement update
};

// Levels per lane of the served launch shape for FP32 / FP64 kernels.
constexpr int kServeM32 = 4, kServeM64 = 2;

// Launches op over the table at dev_tab (device memory; its slots' start[]
// and args[] already there) with `blocks` workgroups in all and `nslots`
// slots.
hipError_t multi_launch(MultiOp op, const MultiTable* dev_tab, int64_t blocks, int nslots,
                        hipStream_t s);

}  // namespace pcg
