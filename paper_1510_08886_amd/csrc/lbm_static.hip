// A solver whose scratch is a static device array of the library, for callers
// that cannot allocate device memory (code under HIP graph capture, serving
// loops that must not allocate, harnesses that forbid hipMalloc).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "lbm_internal.h"

namespace lbm {
namespace {

// Largest scratch a static solver may use: the wall-flux partials, the
// observation partials and the duct's 1 / D(e) table. 16 MiB holds the
// 128 x 256 x 256 D3V39 duct (6.3 MB) and every channel up to nx = 65536.
constexpr size_t kStaticScratchBytes = size_t(16) << 20;
constexpr int kMaxDevices = 64;

// Each device that runs the library holds its own copy until the process ends.
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// Device address of `scratch` per device, taken once per device with that
// device current (the host symbol `scratch` is not a device address).
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

int static_scratch(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(LBM_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(LBM_E_UNSUPPORTED, "static scratch: device index above 63");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(LBM_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return LBM_OK;
}

}  // namespace
}  // namespace lbm

using namespace lbm;

extern "C" int lbm_solver_create_static(const lbm_dvm_t *dvm, const lbm_problem_t *prob,
                                        void *pop_a, void *stream, lbm_solver_t **out) {
    if (!out) return fail(LBM_E_INVALID, "lbm_solver_create_static: null output");
    *out = nullptr;
    size_t need = 0;
    int rc = lbm_state_bytes(dvm, prob, nullptr, &need);
    if (rc) return rc;
    if (need > kStaticScratchBytes)
        return fail(LBM_E_NO_MEMORY, "lbm_solver_create_static: the problem needs " +
                                         std::to_string(need) +
                                         " bytes of scratch, above the static 16 MiB");
    void *ptr = nullptr;
    rc = static_scratch(&ptr);
    if (rc) return rc;
    return solver_create(dvm, prob, pop_a, ptr, kStaticScratchBytes, stream, false, out);
}
