// bddmma_bind_static: a workspace that lives in a static device array of the
// library, for callers that cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "bddmma.h"
#include "solver_internal.hpp"

namespace {

constexpr int kMaxDevices = 64;

// the workspace; each GPU holds its own copy at its own address
static __device__ __align__(256) unsigned char scratch[BDDMMA_STATIC_WORKSPACE_BYTES];

std::mutex g_mu;
void *g_addr[kMaxDevices] = {};                 // device address of `scratch`, per device
const bddmma_solver *g_owner[kMaxDevices] = {}; // solver the array is bound to, per device

}  // namespace

namespace bddmma {

bool static_workspace_held(const bddmma_solver *s, int device)
{
    std::lock_guard<std::mutex> lk(g_mu);
    return device >= 0 && device < kMaxDevices && g_owner[device] == s;
}

void static_workspace_forget(const bddmma_solver *s, int device)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (device >= 0 && device < kMaxDevices && g_owner[device] == s) g_owner[device] = nullptr;
}

}  // namespace bddmma

extern "C" int bddmma_bind_static(bddmma_solver *s, void *hip_stream)
{
    using bddmma::set_error;
    if (!s) return set_error(BDDMMA_ERR_INVALID_ARG, "solver is NULL");
    size_t need = 0;
    int rc = bddmma_workspace_bytes(s, &need);
    if (rc) return rc;
    if (need > BDDMMA_STATIC_WORKSPACE_BYTES)
        return set_error(BDDMMA_ERR_NO_MEMORY,
                         "bddmma_bind_static: the problem needs " + std::to_string(need) +
                             " workspace bytes, above the static workspace of " +
                             std::to_string((size_t)BDDMMA_STATIC_WORKSPACE_BYTES) + " bytes");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(BDDMMA_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return set_error(BDDMMA_ERR_HIP, "device index out of range");
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_addr[dev]) {
            // once per device, with that device current: the host-side name
            // of the array is not a device address
            e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess)
                return set_error(BDDMMA_ERR_HIP, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
            g_addr[dev] = ptr;
        }
        ptr = g_addr[dev];
    }
    rc = bddmma::solver_bind_static(s, ptr, BDDMMA_STATIC_WORKSPACE_BYTES, hip_stream, dev);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    g_owner[dev] = s;
    return BDDMMA_OK;
}
