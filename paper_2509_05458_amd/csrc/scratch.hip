// Device-resident staging for cfmm_eval_static, the evaluation entry point for
// callers that cannot allocate device memory.  The staging lives in a
// file-scope __device__ array, so each GPU that loads the library holds its
// own copy (kStaticScratch complex values, 64 MiB) until the process ends.
// Host code never uses the array's name as an address: static_scratch_init
// resolves each device's copy with hipGetSymbolAddress, once per device, with
// that device current, and static_scratch returns the resolved address.
#include <mutex>

#include "common.hpp"
#include "kernels.hpp"

namespace cfmm {

static __device__ __align__(256) cplx scratch[kStaticScratch];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {nullptr};
}  // namespace

hipError_t static_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_addr[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;   // must be called with `device` current
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_addr[device] = ptr;
    return hipSuccess;
}

cplx* static_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return static_cast<cplx*>(g_addr[device]);
}

}  // namespace cfmm
