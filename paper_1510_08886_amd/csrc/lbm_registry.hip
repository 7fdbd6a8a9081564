// Registry of compiled velocity sets and kernels, and the FP64 finalisation
// of observation sums.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lbm_device.h"

namespace lbm {

const Launch *find_launch_2d(int set_id, Storage st);
const Launch *find_launch_3d(int set_id, Storage st);

int observe_blocks(int64_t nodes) { return (int)blocks_for(nodes); }

// fixed-order sum of partial[n][2]
__global__ __launch_bounds__(256) void k_finalize(const double *partial, int n, double *out) {
    __shared__ double sa[256], sb[256];
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) {
        a += partial[2 * k];
        b += partial[2 * k + 1];
    }
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            sa[threadIdx.x] += sa[threadIdx.x + off];
            sb[threadIdx.x] += sb[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sa[0];
        out[1] = sb[0];
    }
}

// zero fill of a device buffer (used instead of hipMemsetAsync so that the
// launch may also be recorded in a captured graph)
__global__ __launch_bounds__(256) void k_zero(uint32_t *p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

int launch_zero(void *p, size_t bytes, hipStream_t st) {
    if (bytes % 4 != 0 || (uintptr_t)p % 4 != 0)
        return fail(LBM_E_INVALID, "zero fill: 4-byte aligned buffers and sizes only");
    const size_t n = bytes / 4;
    if (n == 0) return LBM_OK;
    const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, st, (uint32_t *)p, n);
    return hip_ok(hipGetLastError(), "zero kernel launch");
}

int launch_finalize(const double *partials, int n, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, partials, n, out);
    return hip_ok(hipGetLastError(), "finalize kernel launch");
}

template <class SET>
static VelSetInfo set_info(const char *name) {
    VelSetInfo v;
    v.name = name;
    v.id = SET::ID;
    v.dim = SET::D;
    v.V = SET::V;
    v.nr = SET::NR;
    for (int p = 0; p < SET::NP; ++p) {
        v.ex.push_back(SET::EX[p]);
        v.ey.push_back(SET::EY[p]);
        v.ez.push_back(SET::EZ[p]);
    }
    return v;
}

const std::vector<VelSetInfo> &velocity_sets() {
    static const std::vector<VelSetInfo> sets = {
        set_info<SetD2V17>("D2V17"), set_info<SetD2V37>("D2V37"), set_info<SetD2V16>("D2V16"),
        set_info<SetD2V33>("D2V33"), set_info<SetD3V39>("D3V39"), set_info<SetD3V15>("D3V15"),
        set_info<SetD2V32>("D2V32"), set_info<SetD3V96>("D3V96"),
    };
    return sets;
}

const Launch *find_launch(int set_id, Storage s) {
    if (const Launch *l = find_launch_2d(set_id, s)) return l;
    return find_launch_3d(set_id, s);
}

}  // namespace lbm
