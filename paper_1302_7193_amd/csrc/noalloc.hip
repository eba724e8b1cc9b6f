// Allocation-free solve: pcg_solve_noalloc runs pcg_solve's kernels with
// their workspace (iteration vectors, partial sums, solver states) in a
// fixed device array of this library instead of a caller-provided buffer,
// for callers that cannot allocate device memory.
//
// The array is a file-scope __device__ variable: every device the library
// runs on holds its own copy for the life of the process.  Host code must
// not use the array's name as a device address (it is a host-side stand-in);
// its device address is looked up once per device with hipGetSymbolAddress
// and that address is what the solve receives.
#include <mutex>
#include <sstream>

#include "problem.h"

namespace pcg {

size_t workspace_bytes(const pcg_problem* P, const pcg_solve_opts& o, int64_t nrhs);
pcg_status solve(pcg_problem* P, const double* b, double* x, void* workspace, size_t ws_bytes,
                 const pcg_solve_opts& o, int64_t nrhs, pcg_result* res, hipStream_t s);

namespace {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_mu;
void* g_addr[kMaxDevices] = {};

// Device address of this device's copy of the array (looked up on the first
// call on that device, with it current), or null with the error set.
void* scratch_address(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("pcg_solve_noalloc: device index out of range");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_addr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            std::ostringstream m;
            m << "pcg_solve_noalloc: hipGetSymbolAddress(scratch): " << hipGetErrorName(e);
            set_error(m.str());
            return nullptr;
        }
        g_addr[dev] = ptr;
    }
    return g_addr[dev];
}

}  // namespace

// Runs with the problem's device current.  The workspace needs nothing
// cleared: every kernel of a solve writes its vectors, partial sums and
// states before reading them.
pcg_status solve_noalloc(pcg_problem* P, const double* b, double* x, const pcg_solve_opts& o0,
                         pcg_result* res, hipStream_t s)
{
    pcg_solve_opts o = o0;
    o.graph_chunk = 0;   // direct launches: instantiating a graph allocates
    o.profile = 0;       // no timing events
    const size_t need = workspace_bytes(P, o, 1);
    if (need > kNoAllocScratchBytes) {
        std::ostringstream m;
        m << "pcg_solve_noalloc: this solve needs " << need << " bytes of workspace; the "
          << "library's fixed scratch holds " << kNoAllocScratchBytes
          << " (use pcg_solve with a workspace)";
        set_error(m.str());
        return PCG_E_NOMEM;
    }
    if (P->pinned_cap < 1) {
        set_error("pcg_solve_noalloc: the problem has no pinned state buffer (internal)");
        return PCG_E_DEVICE;
    }
    void* ws = scratch_address(P->device);
    if (!ws) return PCG_E_DEVICE;
    return solve(P, b, x, ws, kNoAllocScratchBytes, o, 1, res, s);
}

}  // namespace pcg
