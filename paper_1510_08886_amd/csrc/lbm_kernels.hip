// HIP kernels for gfx950: fused pull-stream + diffuse Maxwell wall + BGK
// collision of the modified populations (Eq. nm.8) on 2D channels, plus
// observation, initialisation and population import/export.
//
// Layout in HBM: blocks of 64 consecutive nodes (node n = y * nx + x) with all
// populations of a block together, one contiguous 64-entry run per velocity
// (aos_base). A wavefront covers one block: every store is a whole aligned run
// and every pull load of velocity alpha is one run shifted by the velocity,
// spanning at most two blocks of the source row.
//
// Kernels are specialised per velocity set (lbm_sets.h): integer velocity
// components are compile-time constants, so moments are integer-weighted sums,
// zero components cost nothing, and source offsets come from per-node tables
// of row and column offsets. Velocities come in pairs (e, -e); the even and odd
// parts of the equilibrium and force are formed once per pair.
//
// Arithmetic: the collision works on deviations d = fbar - w rho0 so that the
// moments of a nearly uniform state do not cancel in FP32.
//
// Wall (Eqs. nm.14, nm.15, transformed to fbar): an unknown population at node
// x is rho_eff(e) w (1 - dt/2 g.xi), with rho_eff(e) = A(e) / D(e); A(e) is the
// FP64 sum of the post-collision populations that crossed the wall at element e
// in this streaming step. A step writes, per wall row r < HN and column, the
// FP64 partial of the populations it has just stored that leave through the
// wall next step; the next step sums the partials of its column. The element
// is the column of the fluid node next to the crossing.
#include <hip/hip_runtime.h>

#include <utility>

#include "lbm_node2d.h"

namespace lbm {

// ---------------------------------------------------------------------------
// 2D gather: pull-stream from src with wall slots, in two phases so that the
// loads of one node can be in flight while another node is collided:
//   issue2d    loads the raw stored values of the pull sources; rows outside
//              the channel are clamped so every address is valid;
//   complete2d decodes them to deviations and replaces the values whose source
//              lies outside by the diffuse-wall populations.
// ---------------------------------------------------------------------------
template <class SET, Storage S, bool ALIGNED>
__device__ __forceinline__ void issue2d(const typename St<S>::T *__restrict__ src,
                                        const StepScalars<typename St<S>::R> &s, int i, int j,
                                        typename St<S>::T (&raw)[SET::V]) {
    constexpr int NR = SET::NR, H = SET::H, HN = SET::HN, V = SET::V;
    const int nx = s.nx, ny = s.ny;
    // column offsets (i - k) mod nx for k in [-H, H]
    uint32_t xo[2 * H + 1];
#pragma unroll
    for (int k = -H; k <= H; ++k) xo[k + H] = (uint32_t)wrap_col(i - k, nx, H);
    // source rows j - k clamped into the channel, k in [-HN, HN]
    int rows[2 * HN + 1];
#pragma unroll
    for (int k = -HN; k <= HN; ++k) rows[k + HN] = min(max(j - k, 0), ny - 1);
    if constexpr (NR) raw[0] = src[aos_base<V>((uint32_t)j * nx + i)];
    if constexpr (ALIGNED) {
        // a row is a whole number of blocks: index = row base + column part
        const uint32_t rowstride = (uint32_t)nx * V;
        uint32_t cp[2 * H + 1];
#pragma unroll
        for (int k = 0; k < 2 * H + 1; ++k) cp[k] = (xo[k] >> 6) * (uint32_t)(64 * V) + (xo[k] & 63u);
        for_pairs<SET::NP>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            constexpr int ex = SET::EX[p], ey = SET::EY[p];
            raw[NR + 2 * p] = src[(uint32_t)rows[ey + HN] * rowstride + cp[ex + H] + 64 * (NR + 2 * p)];
            raw[NR + 2 * p + 1] =
                src[(uint32_t)rows[-ey + HN] * rowstride + cp[-ex + H] + 64 * (NR + 2 * p + 1)];
        });
    } else {
        for_pairs<SET::NP>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            constexpr int ex = SET::EX[p], ey = SET::EY[p];
            const uint32_t np_ = (uint32_t)rows[ey + HN] * nx + xo[ex + H];
            const uint32_t nm_ = (uint32_t)rows[-ey + HN] * nx + xo[-ex + H];
            raw[NR + 2 * p] = src[aos_base<V>(np_) + 64 * (NR + 2 * p)];
            raw[NR + 2 * p + 1] = src[aos_base<V>(nm_) + 64 * (NR + 2 * p + 1)];
        });
    }
}

template <class SET, Storage S>
__device__ __forceinline__ void gather2d(const typename St<S>::T *__restrict__ src,
                                         const double *__restrict__ a_cur,
                                         const PairTable<typename St<S>::R> &t,
                                         const StepScalars<typename St<S>::R> &s, int i, int j,
                                         typename St<S>::R (&d)[SET::V]) {
    typename St<S>::T raw[SET::V];
    issue2d<SET, S, false>(src, s, i, j, raw);
    complete2d<SET, S>(raw, a_cur, t, s, i, j, d);
}

// store d[] and, on wall rows, the FP64 partial of what leaves next step
template <class SET, Storage S, bool SRND, bool STREAM = false>
__device__ __forceinline__ void scatter2d(typename St<S>::T *__restrict__ dst,
                                          double *__restrict__ a_next,
                                          const PairTable<typename St<S>::R> &t,
                                          const StepScalars<typename St<S>::R> &s, int i, int j,
                                          const typename St<S>::R (&d)[SET::V], uint32_t step) {
    using T = typename St<S>::T;
    const uint32_t n = (uint32_t)j * s.nx + i;
    T v[SET::V];
    encode_all<SET, S, SRND>(d, t, n, step, v);
    T *out = dst + aos_base<SET::V>(n);
#pragma unroll
    for (int a = 0; a < SET::V; ++a) store_pop<STREAM>(out + 64 * a, v[a]);
    wall_partials2d<SET, S>(v, t, s, i, j, a_next);
}

// One block of 256 threads per tile of 256 consecutive nodes. Each thread
// issues the pull loads of all its velocities before it decodes any of them,
// so a wavefront has its whole gather in flight at once; the wall slots are
// patched after the loads. ALIGNED (nx a multiple of 64) is compiled apart so
// the common case carries no registers of the general index path. Measured on
// MI355X against: a persistent grid with a two-stage register load pipeline
// (occupancy 2), a persistent grid streaming the next tile's gather into LDS
// with global_load_lds (LDS-limited to 8 waves per CU), 64-, 128- and 512-node
// tiles, and register caps for 6, 7 or 8 waves per SIMD.
template <class SET, Storage S, bool ALIGNED, bool STREAM>
__global__ __launch_bounds__(256)
void k_step2d(StepBuffers b, PairTable<typename St<S>::R> t, StepScalars<typename St<S>::R> s,
              uint32_t step) {
    using R = typename St<S>::R;
    using T = typename St<S>::T;
    const uint32_t n = blockIdx.x * 256u + threadIdx.x;
    if (n >= (uint32_t)s.nodes) return;
    const int j = (int)(n / (uint32_t)s.nx);
    const int i = (int)(n - (uint32_t)j * s.nx);
    T raw[SET::V];
    issue2d<SET, S, ALIGNED>((const T *)b.src, s, i, j, raw);
    R d[SET::V];
    complete2d<SET, S>(raw, b.a_cur, t, s, i, j, d);
    relax2d<SET, R>(d, t, s, t.c);
    scatter2d<SET, S, true, STREAM>((T *)b.dst, b.a_next, t, s, i, j, d, step);
}

// ---------------------------------------------------------------------------
// observation: moments of the streamed state, FP64 partial sums per block
// ---------------------------------------------------------------------------
template <class SET, Storage S>
__global__ __launch_bounds__(256) void k_observe2d(const void *src, const double *a_cur,
                                                   double *rho_out, double *u_out, double *partial,
                                                   PairTable<typename St<S>::R> t,
                                                   StepScalars<typename St<S>::R> s) {
    using R = typename St<S>::R;
    using T = typename St<S>::T;
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    double ux_d = 0.0, rho_d = 0.0;
    if (n < (uint32_t)s.nodes) {
        const int j = (int)(n / (uint32_t)s.nx);
        const int i = (int)(n - (uint32_t)j * s.nx);
        R d[SET::V];
        gather2d<SET, S>((const T *)src, a_cur, t, s, i, j, d);
        const auto m = moments2d<SET, R>(d, s, t.c);
        rho_d = s.rho0d + (double)m.drho;
        ux_d = (double)m.ux;
        if (rho_out) rho_out[n] = rho_d;
        if (u_out) {
            u_out[3 * n] = (double)m.ux;
            u_out[3 * n + 1] = (double)m.uy;
            u_out[3 * n + 2] = 0.0;
        }
    }
    block_sum2(ux_d, rho_d, partial);
}

// ---------------------------------------------------------------------------
// init / import / export
// ---------------------------------------------------------------------------
template <class SET, Storage S>
__global__ __launch_bounds__(256) void k_init2d(void *dst, double *a_out, const double *rho_in,
                                                const double *u_in,
                                                PairTable<typename St<S>::R> t,
                                                StepScalars<typename St<S>::R> s, uint32_t step) {
    using R = typename St<S>::R;
    using T = typename St<S>::T;
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (uint32_t)s.nodes) return;
    const int j = (int)(n / (uint32_t)s.nx);
    const int i = (int)(n - (uint32_t)j * s.nx);
    const double rho = rho_in ? rho_in[n] : s.rho0d;
    R ux = 0, uy = 0;
    if (u_in) {
        ux = (R)u_in[3 * n];
        uy = (R)u_in[3 * n + 1];
    }
    R d[SET::V];
    equilibrium_dev<SET, R>(t, s, rho, ux, uy, R(0), d);
    scatter2d<SET, S, false>((T *)dst, a_out, t, s, i, j, d, step);
}

template <class SET, Storage S>
__global__ __launch_bounds__(256) void k_import2d(void *dst, double *a_out, const double *in,
                                                  PairTable<typename St<S>::R> t,
                                                  StepScalars<typename St<S>::R> s, uint32_t step) {
    using R = typename St<S>::R;
    using T = typename St<S>::T;
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (uint32_t)s.nodes) return;
    const int j = (int)(n / (uint32_t)s.nx);
    const int i = (int)(n - (uint32_t)j * s.nx);
    R d[SET::V];
    import_node<SET, R>(in, t, (uint32_t)s.nodes, n, d);
    scatter2d<SET, S, false>((T *)dst, a_out, t, s, i, j, d, step);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <class SET, Storage S>
struct L2 {
    using R = typename St<S>::R;
    static int step(const StepBuffers &b, const void *tab, const void *sc, hipStream_t st,
                    uint32_t stp) {
        const auto &t = *(const PairTable<R> *)tab;
        const auto &s = *(const StepScalars<R> *)sc;
        const dim3 g(blocks_for(s.nodes)), bl(256);
        if (s.aligned_rows && s.stream_stores)
            hipLaunchKernelGGL((k_step2d<SET, S, true, true>), g, bl, 0, st, b, t, s, stp);
        else if (s.aligned_rows)
            hipLaunchKernelGGL((k_step2d<SET, S, true, false>), g, bl, 0, st, b, t, s, stp);
        else
            hipLaunchKernelGGL((k_step2d<SET, S, false, false>), g, bl, 0, st, b, t, s, stp);
        return hip_ok(hipGetLastError(), "step kernel launch");
    }
    static int init(void *dst, double *a_out, const double *rho, const double *u, const void *tab,
                    const void *sc, hipStream_t st, uint32_t stp) {
        const auto &t = *(const PairTable<R> *)tab;
        const auto &s = *(const StepScalars<R> *)sc;
        hipLaunchKernelGGL((k_init2d<SET, S>), dim3(blocks_for(s.nodes)), dim3(256), 0, st, dst,
                           a_out, rho, u, t, s, stp);
        return hip_ok(hipGetLastError(), "init kernel launch");
    }
    static int observe(const void *src, const double *a_cur, const double * /*invd*/, double *rho,
                       double *u, double *partial, const void *tab, const void *sc,
                       hipStream_t st) {
        const auto &t = *(const PairTable<R> *)tab;
        const auto &s = *(const StepScalars<R> *)sc;
        hipLaunchKernelGGL((k_observe2d<SET, S>), dim3(blocks_for(s.nodes)), dim3(256), 0, st,
                           src, a_cur, rho, u, partial, t, s);
        return hip_ok(hipGetLastError(), "observe kernel launch");
    }
    static int exportp(const void *src, double *out, const void *tab, const void *sc,
                       hipStream_t st) {
        const auto &t = *(const PairTable<R> *)tab;
        const auto &s = *(const StepScalars<R> *)sc;
        hipLaunchKernelGGL((k_export<SET, S>), dim3(blocks_for(s.nodes)), dim3(256), 0, st, src,
                           out, t, s);
        return hip_ok(hipGetLastError(), "export kernel launch");
    }
    static int importp(void *dst, double *a_out, const double *in, const void *tab, const void *sc,
                       hipStream_t st, uint32_t stp) {
        const auto &t = *(const PairTable<R> *)tab;
        const auto &s = *(const StepScalars<R> *)sc;
        hipLaunchKernelGGL((k_import2d<SET, S>), dim3(blocks_for(s.nodes)), dim3(256), 0, st,
                           dst, a_out, in, t, s, stp);
        return hip_ok(hipGetLastError(), "import kernel launch");
    }
    static constexpr Launch table{&step, &init, &observe, &exportp, &importp};
};

#define LBM_2D(SET)                                                           \
    {SET::ID, Storage::F64, &L2<SET, Storage::F64>::table},                   \
        {SET::ID, Storage::F32, &L2<SET, Storage::F32>::table},               \
        {SET::ID, Storage::F32RAW, &L2<SET, Storage::F32RAW>::table},         \
        {SET::ID, Storage::F16DEV, &L2<SET, Storage::F16DEV>::table}

const Launch *find_launch_2d(int set_id, Storage st) {
    static const Entry entries[] = {
        LBM_2D(SetD2V17), LBM_2D(SetD2V37), LBM_2D(SetD2V16), LBM_2D(SetD2V33), LBM_2D(SetD2V32),
    };
    for (const auto &e : entries)
        if (e.id == set_id && e.s == st) return e.l;
    return nullptr;
}

}  // namespace lbm
