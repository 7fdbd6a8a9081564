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

#include "lbm_device.h"

namespace lbm {

// ---------------------------------------------------------------------------
// per-node collision on deviations (2D channel, g along x): d[] in/out
// ---------------------------------------------------------------------------
template <typename R>
struct Moments2D {
    R drho, rho, ux, uy, sxx, sxy, syy;
};

template <class SET, typename R>
__device__ __forceinline__ Moments2D<R> moments2d(const R (&d)[SET::V], const StepScalars<R> &s,
                                                  R c) {
    constexpr int NR = SET::NR;
    R drho = NR ? d[0] : R(0);
    R jx = 0, jy = 0, sxx = 0, syy = 0, sxy = 0;
    for_pairs<SET::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int ex = SET::EX[p], ey = SET::EY[p];
        const R dp = d[NR + 2 * p], dm = d[NR + 2 * p + 1];
        const R sum = dp + dm, dif = dp - dm;
        drho += sum;
        jx = addk<ex>(jx, dif);
        jy = addk<ey>(jy, dif);
        sxx = addk<ex * ex>(sxx, sum);
        syy = addk<ey * ey>(syy, sum);
        sxy = addk<ex * ey>(sxy, sum);
    });
    Moments2D<R> m;
    const R c2 = c * c;
    m.drho = drho;
    m.rho = s.rho0 + drho;
    const R inv = R(1) / m.rho;
    m.ux = fma(s.half_dt_g[0], m.rho, jx * c) * inv;
    m.uy = jy * c * inv;
    m.sxx = sxx * c2;
    m.syy = syy * c2;
    m.sxy = sxy * c2;
    return m;
}

template <class SET, typename R>
__device__ __forceinline__ void relax2d(R (&d)[SET::V], const PairTable<R> &t,
                                        const StepScalars<R> &s, R c) {
    constexpr int NR = SET::NR;
    const auto m = moments2d<SET, R>(d, s, c);
    const R drho = m.drho, rho = m.rho, ux = m.ux, uy = m.uy;
    const R gx = s.g[0];
    // a2 = Pi(f) - rho I from fbar by inverting Eq. nm.7 (deviation form)
    const R hr = s.h * rho;
    const R htr = hr * s.tau;
    const R a2xx = (m.sxx - drho + hr * ux * ux + R(2) * htr * gx * ux) * s.inv1h;
    const R a2yy = (m.syy - drho + hr * uy * uy) * s.inv1h;
    const R a2xy = (m.sxy + hr * ux * uy + htr * gx * uy) * s.inv1h;
    const R tra2 = a2xx + a2yy;
    const R c2 = c * c;
    const R qxx = a2xx * c2, qyy = a2yy * c2, qxy = a2xy * c2;   // a2 : xi xi
    const R hxc = a2xx * gx * c, hyc = a2xy * gx * c;              // (a2 g) . xi
    const R uxc = ux * c, uyc = uy * c;
    const R gxc = gx * c;
    const R u2 = ux * ux + uy * uy;
    const R u2_3 = R(3) * u2;
    const R ug = ux * gx;
    const R tr = s.tau * rho;
    const R trgxc = tr * gxc;
    const R half_tau = R(0.5) * s.tau;
    const R rc2 = rho * s.cn[2], rc3 = rho * s.cn[3], rc4 = rho * s.cn[4];
    const R om = s.omega;
    const R even0 = drho - tr * ug;   // part of the even term shared by all velocities
    if constexpr (NR) {
        // rest velocity: P2 = -u2, P4 = 3 u2^2, no odd part
        const R even = fma(rc2, -u2, fma(rc4, u2_3 * u2, even0));
        d[0] = fma(om, fma(t.w0, even, -d[0]), d[0]);
    }
    for_pairs<SET::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int ex = SET::EX[p], ey = SET::EY[p];
        const R ue = lin2<ex, ey>(uxc, uyc);
        const R ue2 = ue * ue;
        const R P2 = ue2 - u2;
        const R P3 = ue * (ue2 - u2_3);
        const R P4 = fma(ue, P3, -u2_3 * P2);
        // even: drho + rho (P2/2 + P4/24) + tau rho ((g.xi)(u.xi) - u.g)
        R even = fma(rc2, P2, fma(rc4, P4, even0));
        R odd = fma(rc3, P3, rho * ue);
        if constexpr (ex != 0) {
            even = fma(mulk<ex>(trgxc), ue, even);
            // tau F, odd part: (g.xi) [tau rho + tau/2 (a2 : xi xi - tr a2)]
            const R q = lin3<ex * ex, ey * ey, 2 * ex * ey>(qxx, qyy, qxy);
            odd = fma(mulk<ex>(gxc), fma(half_tau, q - tra2, tr), odd);
        }
        // - tau (a2 g) . xi
        if constexpr (ex != 0 || ey != 0) odd = fma(-s.tau, lin2<ex, ey>(hxc, hyc), odd);
        const R w = t.w[p];
        R &dp = d[NR + 2 * p];
        R &dm = d[NR + 2 * p + 1];
        dp = fma(om, fma(w, even + odd, -dp), dp);
        dm = fma(om, fma(w, even - odd, -dm), dm);
    });
}

// ---------------------------------------------------------------------------
// 2D gather: pull-stream from src with wall slots, in two phases so that the
// loads of one node can be in flight while another node is collided:
//   issue2d    loads the raw stored values of the pull sources; rows outside
//              the channel are clamped so every address is valid;
//   complete2d decodes them to deviations and replaces the values whose source
//              lies outside by the diffuse-wall populations.
// ---------------------------------------------------------------------------
template <class SET, Storage S>
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
    if (s.aligned_rows) {
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
__device__ __forceinline__ void complete2d(const typename St<S>::T (&raw)[SET::V],
                                           const double *__restrict__ a_cur,
                                           const PairTable<typename St<S>::R> &t,
                                           const StepScalars<typename St<S>::R> &s, int i, int j,
                                           typename St<S>::R (&d)[SET::V]) {
    using R = typename St<S>::R;
    constexpr int NR = SET::NR, HN = SET::HN;
    const int nx = s.nx, ny = s.ny;
    if constexpr (NR) d[0] = decode_dev<S>(raw[0], t.wr00);
    for_pairs<SET::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        d[NR + 2 * p] = decode_dev<S>(raw[NR + 2 * p], t.wr0[p]);
        d[NR + 2 * p + 1] = decode_dev<S>(raw[NR + 2 * p + 1], t.wr0[p]);
    });
    if ((j < HN) || (j >= ny - HN)) {
        // rho_eff of this column on each face from the FP64 partials
        double alo = 0.0, ahi = 0.0;
#pragma unroll
        for (int r = 0; r < HN; ++r) {
            alo += a_cur[r * nx + i];
            ahi += a_cur[(HN + r) * nx + i];
        }
        const double rlo = alo * s.invD[0], rhi = ahi * s.invD[1];
        // wall population w (rho_eff (1 - dt/2 g.xi)) as a deviation from w rho0
        const double rho0 = s.rho0d, hgc = s.hgc;
        for_pairs<SET::NP>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            constexpr int ex = SET::EX[p], ey = SET::EY[p];
            if constexpr (ey != 0) {
                const double wd = (double)t.w[p];
                int js = j - ey;
                if (js < 0 || js >= ny) {
                    const double re = js < 0 ? rlo : rhi;
                    d[NR + 2 * p] = (R)(wd * (re * (1.0 - hgc * ex) - rho0));
                }
                js = j + ey;
                if (js < 0 || js >= ny) {
                    const double re = js < 0 ? rlo : rhi;
                    d[NR + 2 * p + 1] = (R)(wd * (re * (1.0 + hgc * ex) - rho0));
                }
            }
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
    issue2d<SET, S>(src, s, i, j, raw);
    complete2d<SET, S>(raw, a_cur, t, s, i, j, d);
}

// store d[] and, on wall rows, the FP64 partial of what leaves next step
template <class SET, Storage S, bool SRND>
__device__ __forceinline__ void scatter2d(typename St<S>::T *__restrict__ dst,
                                          double *__restrict__ a_next,
                                          const PairTable<typename St<S>::R> &t,
                                          const StepScalars<typename St<S>::R> &s, int i, int j,
                                          const typename St<S>::R (&d)[SET::V], uint32_t step) {
    using T = typename St<S>::T;
    constexpr int NR = SET::NR, HN = SET::HN;
    const int nx = s.nx, ny = s.ny;
    const uint32_t n = (uint32_t)j * nx + i;
    T v[SET::V];
    encode_all<SET, S, SRND>(d, t, n, step, v);
    T *out = dst + aos_base<SET::V>(n);
#pragma unroll
    for (int a = 0; a < SET::V; ++a) out[64 * a] = v[a];
    if (j < HN || j >= ny - HN) {
        double lo = 0.0, hi = 0.0;
        for_pairs<SET::NP>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            constexpr int ey = SET::EY[p];
            if constexpr (ey != 0) {
                const double vp = stored_part<S>(v[NR + 2 * p], t.wr0[p]);
                const double vm = stored_part<S>(v[NR + 2 * p + 1], t.wr0[p]);
                if (j + ey < 0) lo += vp;
                if (j - ey < 0) lo += vm;
                if (j + ey >= ny) hi += vp;
                if (j - ey >= ny) hi += vm;
            }
        });
        if (j < HN) a_next[j * nx + i] = s.kA[0][j] + lo;
        if (j >= ny - HN) a_next[(HN + (ny - 1 - j)) * nx + i] = s.kA[1][ny - 1 - j] + hi;
    }
}

// One block of 256 threads per tile of 256 consecutive nodes. Each thread
// issues the pull loads of all its velocities before it decodes any of them,
// so a wavefront has its whole gather in flight at once; the wall slots are
// patched after the loads. (Measured on MI355X: this beats a persistent grid
// with a two-stage load pipeline, whose second register buffer halves the
// occupancy, and 128- or 512-node tiles.)
template <class SET, Storage S>
__global__ __launch_bounds__(256) void k_step2d(StepBuffers b, PairTable<typename St<S>::R> t,
                                                StepScalars<typename St<S>::R> s, uint32_t step) {
    using R = typename St<S>::R;
    using T = typename St<S>::T;
    const uint32_t n = blockIdx.x * 256u + threadIdx.x;
    if (n >= (uint32_t)s.nodes) return;
    const int j = (int)(n / (uint32_t)s.nx);
    const int i = (int)(n - (uint32_t)j * s.nx);
    T raw[SET::V];
    issue2d<SET, S>((const T *)b.src, s, i, j, raw);
    R d[SET::V];
    complete2d<SET, S>(raw, b.a_cur, t, s, i, j, d);
    relax2d<SET, R>(d, t, s, t.c);
    scatter2d<SET, S, true>((T *)b.dst, b.a_next, t, s, i, j, d, step);
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
        hipLaunchKernelGGL((k_step2d<SET, S>), dim3(blocks_for(s.nodes)), dim3(256), 0, st, b, t,
                           s, stp);
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
    static int observe(const void *src, const double *a_cur, double *rho, double *u,
                       double *partial, const void *tab, const void *sc, hipStream_t st) {
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
        LBM_2D(SetD2V17), LBM_2D(SetD2V37), LBM_2D(SetD2V16), LBM_2D(SetD2V33),
    };
    for (const auto &e : entries)
        if (e.id == set_id && e.s == st) return e.l;
    return nullptr;
}

}  // namespace lbm
