// Poisson solve that allocates nothing and takes no workspace argument: the
// work fields and per-call state live in a fixed device array of this
// library, for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops, harnesses that forbid allocation).
//
// The array is a file-scope __device__ object, so every GPU the library
// runs on holds its own copy until the process ends.  Host code never uses
// the array's name as an address (on the host it is only a stand-in for
// the symbol): the first call on a device, with that device current,
// resolves the device address with hipGetSymbolAddress and keeps it per
// device; kernels then receive that address like any workspace.
#include <mutex>

#include "ibs_internal.h"

namespace ibs {

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;   // 64 MiB per device
static_assert(NOALLOC_SCRATCH_BYTES == IBS_NOALLOC_SCRATCH_BYTES, "scratch size and the ABI disagree");

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;

// Device address of `scratch` on the current device, resolved once per
// device; nullptr (and the error set) when the symbol cannot be resolved.
static void *scratch_on_current_device()
{
    static std::mutex mu;
    static void *addr[MAX_DEVICES] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        set_error(std::string("solve_poisson_noalloc: no current device: ") + hipGetErrorString(e));
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error(std::string("solve_poisson_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
            return nullptr;
        }
        addr[dev] = ptr;
    }
    return addr[dev];
}

}  // namespace ibs

using namespace ibs;

extern "C" ibs_status solve_poisson_noalloc(ibs_plan plan, const double *b, double *phi,
                                            ibs_solve_info *info, void *stream)
{
    if (!plan) { set_error("plan is NULL"); return IBS_ERR_INVALID_ARG; }
    size_t work_bytes = 0;
    ibs_status st = solver_plan_bytes(plan, IBS_OP_POISSON, 1, nullptr, &work_bytes);
    if (st != IBS_OK) return st;
    if (work_bytes > NOALLOC_SCRATCH_BYTES) {
        set_error("solve_poisson_noalloc: the grid needs " + std::to_string(work_bytes) +
                  " bytes of workspace, more than the library's fixed " +
                  std::to_string(NOALLOC_SCRATCH_BYTES) + "-byte scratch; use solve_poisson");
        return IBS_ERR_WORKSPACE_TOO_SMALL;
    }
    void *work = scratch_on_current_device();
    if (!work) return IBS_ERR_HIP;
    // every word of the workspace that a solve reads it has written earlier
    // in the same call, so nothing needs clearing between calls
    return solve_poisson(plan, b, phi, work, work_bytes, info, stream);
}
