// Per-call device work space, ordered on the caller's stream.
//
// Entry points that need scratch memory beyond their inputs and outputs (the
// Gram records of the matching step, the buffers of a Poisson solve) take it
// from a library-owned memory pool with hipMallocFromPoolAsync on the call's
// stream and hand it back with hipFreeAsync on the same stream after the last
// launch that uses it.  Two calls on different streams therefore never share
// work space, a plan stays read-only after creation, and the pool keeps the
// memory for reuse (release threshold: never), so a steady stream of calls
// does not reach the device allocator.
#include <stdint.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>

#include "internal.h"

namespace fc2d {

namespace {
std::mutex g_pool_mu;
std::map<int, hipMemPool_t> g_pools;   // one pool per device, kept for the process's life

int pool_for_current_device(hipMemPool_t* out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
        return FC2D_E_HIP;
    }
    std::lock_guard<std::mutex> lk(g_pool_mu);
    auto it = g_pools.find(dev);
    if (it != g_pools.end()) {
        *out = it->second;
        return FC2D_OK;
    }
    hipMemPoolProps props;
    memset(&props, 0, sizeof props);
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t pool = nullptr;
    if ((e = hipMemPoolCreate(&pool, &props)) != hipSuccess) {
        set_error(std::string("hipMemPoolCreate: ") + hipGetErrorString(e));
        return FC2D_E_HIP;
    }
    uint64_t keep = UINT64_MAX;
    if ((e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep)) != hipSuccess) {
        (void)hipMemPoolDestroy(pool);
        set_error(std::string("hipMemPoolSetAttribute: ") + hipGetErrorString(e));
        return FC2D_E_HIP;
    }
    g_pools[dev] = pool;
    *out = pool;
    return FC2D_OK;
}
}  // namespace

int ws_alloc(size_t bytes, hipStream_t s, void** p) {
    *p = nullptr;
    hipMemPool_t pool;
    int st = pool_for_current_device(&pool);
    if (st) return st;
    hipError_t e = hipMallocFromPoolAsync(p, bytes ? bytes : 256, pool, s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        set_error(std::string("device work space (") + std::to_string(bytes) + " bytes): " + hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? FC2D_E_NOMEM : FC2D_E_HIP;
    }
    return FC2D_OK;
}

int ws_free(void* p, hipStream_t s) {
    if (!p) return FC2D_OK;
    hipError_t e = hipFreeAsync(p, s);
    if (e != hipSuccess) {
        set_error(std::string("hipFreeAsync: ") + hipGetErrorString(e));
        return FC2D_E_HIP;
    }
    return FC2D_OK;
}

}  // namespace fc2d
