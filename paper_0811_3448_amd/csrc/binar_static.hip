// Allocation-free sort (binar_sort_static): the same launch sequence as
// binar_sort_async, with its scratch in a fixed per-device array of the
// library instead of a caller workspace or the growing pool.
//
// `scratch` below is a device variable.  In host code its name is only a
// host-side stand-in for it, so it is never passed anywhere: its device
// address is looked up once per device with hipGetSymbolAddress (with that
// device current) and that address is what the kernels receive.
#include <hip/hip_runtime.h>

#include <mutex>

#include "binar.h"
#include "binar_host.h"

namespace binar {
namespace {

__device__ __align__(256) char scratch[BINAR_STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_static_mu;
void *g_static_ptr[MAX_DEVICES];  // device address of `scratch`, per device

int static_scratch(int dev, void **out) {
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *p = nullptr;
        BINAR_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || (reinterpret_cast<uintptr_t>(p) & (ALIGN - 1))) return hip_fail("hipGetSymbolAddress", hipErrorUnknown);
        g_static_ptr[dev] = p;
    }
    *out = g_static_ptr[dev];
    return BINAR_OK;
}

// No timing events while this call enqueues: creating them could allocate.
struct NoEvents {
    bool saved;
    NoEvents() : saved(t_capturing) { t_capturing = true; }
    ~NoEvents() { t_capturing = saved; }
};

}  // namespace
}  // namespace binar

extern "C" int binar_sort_static(void *keys, uint32_t key_bytes, uint64_t n, uint32_t *payload, void *stream) {
    using namespace binar;
    if (key_bytes != 4 && key_bytes != 8 && key_bytes != 16) return BINAR_EINVAL;
    if (n > BINAR_MAX_KEYS) return BINAR_ERANGE;
    if (n < 2) return BINAR_OK;  // base case: nothing to order
    const size_t need = binar_workspace_bytes(key_bytes, n, payload != nullptr, 1, nullptr);
    if (need == 0) return BINAR_EINVAL;
    if (need > (size_t)BINAR_STATIC_SCRATCH_BYTES) return BINAR_ENOMEM;
    int dev = 0;
    BINAR_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return hip_fail("binar_sort_static: device index", hipErrorInvalidDevice);
    void *ws = nullptr;
    if (int rc = static_scratch(dev, &ws)) return rc;
    NoEvents guard;
    return binar_sort_async(keys, key_bytes, n, payload, stream, ws, (size_t)BINAR_STATIC_SCRATCH_BYTES);
}
