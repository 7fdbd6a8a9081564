// Measurement aid, not part of the method: a plain streaming copy, the
// practical bandwidth ceiling that the HBM-bound step kernels are compared with
// (next to the 8 TB/s peak of the part).
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "lbm_internal.h"

using namespace lbm;

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// One 16-byte vector per thread, each byte read once and written once, stores
// non-temporal. On MI355X this was the fastest of the copies measured (one
// vector per thread with plain stores, two per thread, grid-stride loops over
// 2048 to 32768 blocks): 6.35 TB/s for 1.3 GB each way.
__global__ __launch_bounds__(256) void k_stream_copy(const u32x4 *__restrict__ src,
                                                     u32x4 *__restrict__ dst, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(src[i], dst + i);
}

}  // namespace

extern "C" int lbm_stream_copy(const void *src, void *dst, size_t bytes, void *stream) {
    if (!src || !dst || bytes % 16 != 0 || (uintptr_t)src % 16 != 0 || (uintptr_t)dst % 16 != 0)
        return fail(LBM_E_INVALID,
                    "lbm_stream_copy: need 16-byte aligned src and dst and bytes a multiple of 16");
    const size_t n = bytes / 16;
    if (n == 0) return LBM_OK;
    const size_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffffu) return fail(LBM_E_INVALID, "lbm_stream_copy: too many bytes");
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       (const u32x4 *)src, (u32x4 *)dst, n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(LBM_E_DEVICE, std::string("lbm_stream_copy: ") + hipGetErrorString(e));
    return LBM_OK;
}

// Event-to-event duration of individual lbm_run calls on the solver's stream.
extern "C" int lbm_time_launches(lbm_solver_t *h, void *stream, int n, int steps_per_launch,
                                 int system_scope, float *ms_out) {
    if (!h || n < 1 || n > 100000 || steps_per_launch < 1 || !ms_out)
        return fail(LBM_E_INVALID, "lbm_time_launches: bad arguments");
    const hipStream_t st = (hipStream_t)stream;
    const unsigned flags = system_scope ? hipEventReleaseToSystem : hipEventDefault;
    std::vector<hipEvent_t> ev(n + 1, nullptr);
    hipError_t e = hipSuccess;
    for (auto &x : ev)
        if (e == hipSuccess) e = hipEventCreateWithFlags(&x, flags);
    int rc = LBM_OK;
    if (e == hipSuccess) e = hipEventRecord(ev[0], st);
    for (int k = 0; k < n && e == hipSuccess && rc == LBM_OK; ++k) {
        rc = lbm_run(h, steps_per_launch);
        if (rc == LBM_OK) e = hipEventRecord(ev[k + 1], st);
    }
    if (e == hipSuccess && rc == LBM_OK) e = hipEventSynchronize(ev[n]);
    for (int k = 0; k < n && e == hipSuccess && rc == LBM_OK; ++k)
        e = hipEventElapsedTime(&ms_out[k], ev[k], ev[k + 1]);
    for (auto &x : ev)
        if (x) (void)hipEventDestroy(x);
    if (rc) return rc;
    if (e != hipSuccess)
        return fail(LBM_E_DEVICE, std::string("lbm_time_launches: ") + hipGetErrorString(e));
    return LBM_OK;
}
