// HIP kernels for gfx950: fused pull-stream + diffuse Maxwell wall + BGK
// collision of the modified populations (Eq. nm.8), observation, init and
// population import/export.
//
// Layout in HBM: structure of arrays, f[alpha][z][y][x] with x fastest and an
// alpha-plane stride padded to 64 elements. A wavefront covers 64 consecutive
// nodes of one row, so every load of population alpha is one contiguous
// (shifted by e_x) 64-element run and every store is aligned and coalesced.
//
// Arithmetic: the collision works on deviations d = fbar - w rho0 so that the
// moments of a nearly uniform state do not cancel in FP32. Velocities come in
// pairs (e, -e); even and odd parts of the equilibrium and force are formed
// once per pair.
//
// Wall (Eqs. nm.14, nm.15, transformed to fbar): an unknown population at node
// x is rho_eff(e) w (1 - dt/2 g.xi), with rho_eff(e) = A(e) / D(e), where A(e)
// is the FP64 sum of the post-collision populations that crossed the wall at
// element e in this streaming step. A step writes, per wall row r < halo and
// column, the FP64 partial of the populations it has just stored that will
// leave through the wall next step; the next step sums the halo partials of
// its column. Element = column of the fluid node next to the crossing.
#include <hip/hip_runtime.h>

#include "lbm_internal.h"

namespace lbm {

// ---------------------------------------------------------------------------
// storage traits: T is the stored type, R the arithmetic type. The collision
// always sees the deviation d = fbar - w rho0.
//   F64    : fbar in double
//   F32    : d in float
//   F32RAW : fbar in float
//   F16DEV : d / (w rho0) in half, stochastic rounding
// ---------------------------------------------------------------------------
template <Storage S>
struct St;
template <>
struct St<Storage::F64> {
    using T = double;
    using R = double;
};
template <>
struct St<Storage::F32> {
    using T = float;
    using R = float;
};
template <>
struct St<Storage::F32RAW> {
    using T = float;
    using R = float;
};
template <>
struct St<Storage::F16DEV> {
    using T = _Float16;
    using R = float;
};

// PCG-family integer hash (Jarzynski & Olano, "Hash Functions for GPU
// Rendering", JCGT 2020): one 32-bit output per 32-bit input.
__device__ __forceinline__ uint32_t pcg_hash(uint32_t v) {
    const uint32_t state = v * 747796405u + 2891336453u;
    const uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
    return (word >> 22u) ^ word;
}

// Stochastic rounding of a float to half on the magnitude: add 13 random bits
// below the half mantissa and truncate them. Exact in the half normal range;
// below it (|x| < 2^-14) the final conversion rounds to nearest.
__device__ __forceinline__ _Float16 sr_half(float x, uint32_t rnd13) {
    uint32_t b = __float_as_uint(x);
    b = (b + (rnd13 & 0x1FFFu)) & ~0x1FFFu;
    return (_Float16)__uint_as_float(b);
}

template <Storage S>
__device__ __forceinline__ typename St<S>::R decode_dev(typename St<S>::T v,
                                                         typename St<S>::R wr0) {
    using R = typename St<S>::R;
    if constexpr (S == Storage::F16DEV)
        return wr0 * (R)v;
    else if constexpr (S == Storage::F32)
        return v;
    else
        return (R)v - wr0;
}

// SRND selects stochastic rounding for half storage (time steps); init and
// import round to nearest so that an exported state re-imports bit-exactly.
template <Storage S, bool SRND>
__device__ __forceinline__ typename St<S>::T encode_dev(typename St<S>::R d,
                                                         typename St<S>::R wr0,
                                                         typename St<S>::R inv_wr0,
                                                         uint32_t rnd) {
    using T = typename St<S>::T;
    if constexpr (S == Storage::F16DEV && SRND)
        return sr_half(d * inv_wr0, rnd);
    else if constexpr (S == Storage::F16DEV)
        return (T)(d * inv_wr0);
    else if constexpr (S == Storage::F32)
        return (T)d;
    else
        return (T)(d + wr0);
}

// exact FP64 value of a stored population
template <Storage S>
__device__ __forceinline__ double stored_value(typename St<S>::T v, double wrd) {
    if constexpr (S == Storage::F16DEV)
        return wrd * (1.0 + (double)(float)v);
    else if constexpr (S == Storage::F32)
        return wrd + (double)v;
    else
        return (double)v;
}

// per-node random stream for stochastic rounding: one 32-bit word per pair
__device__ __forceinline__ uint32_t node_key(int64_t n, uint32_t step) {
    return pcg_hash((uint32_t)n ^ pcg_hash(step ^ ((uint32_t)(n >> 32) * 0x9E3779B9u)));
}

__device__ __forceinline__ int wrap_sub(int i, int m, int nx) {
    // i in [0, nx), m in [0, nx): (i - m) mod nx
    int r = i - m;
    return r < 0 ? r + nx : r;
}

__device__ __forceinline__ int64_t remap_block(int64_t b, int64_t nb) {
    // consecutive blocks are dispatched round-robin over the 8 XCDs; give each
    // XCD a contiguous range of tiles so its L2 sees neighbouring rows
    int64_t q = nb / 8, r = nb % 8;
    int64_t x = b % 8, k = b / 8;
    return x * q + (x < r ? x : r) + k;
}

// ---------------------------------------------------------------------------
// per-node collision on deviations (2D): d[] in/out
// ---------------------------------------------------------------------------
template <typename R, int V, int NH>
struct Collide2D {
    static constexpr int NR = V & 1;
    static constexpr int NP = V / 2;

    // returns (rho, ux, uy) of the pre-collision state
    __device__ __forceinline__ static void moments(const R (&d)[V], const PairTable<R> &t,
                                                   const StepScalars<R> &s, R &drho, R &rho,
                                                   R &ux, R &uy, R &sxx, R &sxy, R &syy) {
        drho = NR ? d[0] : R(0);
        R jx = 0, jy = 0;
        sxx = 0, sxy = 0, syy = 0;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const R dp = d[NR + 2 * p], dm = d[NR + 2 * p + 1];
            const R sum = dp + dm, dif = dp - dm;
            drho += sum;
            jx = fma(dif, t.xi[p][0], jx);
            jy = fma(dif, t.xi[p][1], jy);
            sxx = fma(sum, t.qq[p][0], sxx);
            syy = fma(sum, t.qq[p][1], syy);
            sxy = fma(sum, t.qq[p][3], sxy);
        }
        rho = s.rho0 + drho;
        const R inv = R(1) / rho;
        ux = (jx + s.half_dt_g[0] * rho) * inv;
        uy = (jy + s.half_dt_g[1] * rho) * inv;
    }

    __device__ __forceinline__ static void relax(R (&d)[V], const PairTable<R> &t,
                                                 const StepScalars<R> &s) {
        R drho, rho, ux, uy, sxx, sxy, syy;
        moments(d, t, s, drho, rho, ux, uy, sxx, sxy, syy);
        const R gx = s.g[0], gy = s.g[1];
        // a2 = Pi(f) - rho I from fbar by inverting Eq. nm.7 (deviation form)
        const R hr = s.h * rho;
        const R htr = hr * s.tau;
        R a2xx = (sxx - drho + hr * ux * ux + R(2) * htr * gx * ux) * s.inv1h;
        R a2yy = (syy - drho + hr * uy * uy + R(2) * htr * gy * uy) * s.inv1h;
        R a2xy = (sxy + hr * ux * uy + htr * (gx * uy + gy * ux)) * s.inv1h;
        const R tra2 = a2xx + a2yy;
        // a2 . g
        const R hvx = a2xx * gx + a2xy * gy;
        const R hvy = a2xy * gx + a2yy * gy;
        const R u2 = ux * ux + uy * uy;
        const R ug = ux * gx + uy * gy;
        const R tr = s.tau * rho;
        const R half_tau = R(0.5) * s.tau;
        const R c2 = s.cn[2], c3 = s.cn[3], c4 = s.cn[4], c5 = s.cn[5];
        const R om = s.omega;
        // rest velocity: xi = 0
        if constexpr (NR) {
            // P2 = -u2, P4 = 3 u2^2, odd terms vanish; force: -tau rho u.g
            const R even = drho + rho * (c2 * (-u2) + c4 * (R(3) * u2 * u2)) - tr * ug;
            const R deq = t.w0 * even;
            d[0] = fma(om, deq - d[0], d[0]);
        }
        (void)c5;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const R xx = t.xi[p][0], xy = t.xi[p][1];
            const R ue = fma(ux, xx, uy * xy);
            const R ge = fma(gx, xx, gy * xy);
            const R ue2 = ue * ue;
            const R P2 = ue2 - u2;
            R even = drho;
            R odd = ue;
            if constexpr (NH >= 2) even = fma(rho * c2, P2, even);
            R P3 = 0;
            if constexpr (NH >= 3) {
                P3 = ue * (ue2 - R(3) * u2);
                odd = fma(c3, P3, odd);
            }
            if constexpr (NH >= 4) {
                const R P4 = fma(ue, P3, -R(3) * u2 * P2);
                even = fma(rho * c4, P4, even);
            }
            odd = rho * odd;
            // force (Eq. nm.4): tau F / w = tau rho ge + tau rho (ge ue - u.g)
            //   + tau/2 [ge (a2 : xi xi - tr a2) - 2 (a2 g) . xi]
            even = fma(tr, ge * ue - ug, even);
            const R q = fma(a2xx, t.qq[p][0], fma(a2yy, t.qq[p][1], R(2) * a2xy * t.qq[p][3]));
            const R hxi = fma(hvx, xx, hvy * xy);
            odd = fma(ge, fma(half_tau, q - tra2, tr), odd);
            odd = fma(-s.tau, hxi, odd);
            const R w = t.w[p];
            const R deqp = w * (even + odd);
            const R deqm = w * (even - odd);
            R &dp = d[NR + 2 * p];
            R &dm = d[NR + 2 * p + 1];
            dp = fma(om, deqp - dp, dp);
            dm = fma(om, deqm - dm, dm);
        }
    }
};

// ---------------------------------------------------------------------------
// 2D gather: pull-stream from src with wall slots
// ---------------------------------------------------------------------------
template <Storage S, int V>
__device__ __forceinline__ void gather2d(const typename St<S>::T *__restrict__ src,
                                         const double *__restrict__ a_cur,
                                         const PairTable<typename St<S>::R> &t,
                                         const StepScalars<typename St<S>::R> &s, int i, int j,
                                         typename St<S>::R (&d)[V]) {
    using R = typename St<S>::R;
    constexpr int NR = V & 1, NP = V / 2;
    const int nx = s.nx, ny = s.ny, H = s.halo;
    const int64_t plane = s.plane;
    const bool near = (j < H) || (j >= ny - H);
    if constexpr (NR) d[0] = decode_dev<S>(src[(int64_t)j * nx + i], t.wr00);
    if (!near) {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int ey = t.ey[p];
            const int64_t ap = (int64_t)(NR + 2 * p) * plane;
            const int64_t am = ap + plane;
            d[NR + 2 * p] = decode_dev<S>(src[ap + (int64_t)(j - ey) * nx + wrap_sub(i, t.exm[p], nx)],
                                          t.wr0[p]);
            d[NR + 2 * p + 1] = decode_dev<S>(
                src[am + (int64_t)(j + ey) * nx + wrap_sub(i, t.exmn[p], nx)], t.wr0[p]);
        }
    } else {
        // rho_eff of this column on each face from the FP64 partials
        double alo = 0.0, ahi = 0.0;
        for (int r = 0; r < H; ++r) {
            alo += a_cur[(int64_t)r * nx + i];
            ahi += a_cur[(int64_t)(H + r) * nx + i];
        }
        const double rlo = alo * s.invD[0], rhi = ahi * s.invD[1];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int ey = t.ey[p];
            const int64_t ap = (int64_t)(NR + 2 * p) * plane;
            const int64_t am = ap + plane;
            int js = j - ey;
            if (js >= 0 && js < ny) {
                d[NR + 2 * p] = decode_dev<S>(src[ap + (int64_t)js * nx + wrap_sub(i, t.exm[p], nx)],
                                              t.wr0[p]);
            } else {
                const double re = js < 0 ? rlo : rhi;
                d[NR + 2 * p] = (R)(re * t.shape_p[p] - t.wrd[p]);
            }
            js = j + ey;
            if (js >= 0 && js < ny) {
                d[NR + 2 * p + 1] = decode_dev<S>(
                    src[am + (int64_t)js * nx + wrap_sub(i, t.exmn[p], nx)], t.wr0[p]);
            } else {
                const double re = js < 0 ? rlo : rhi;
                d[NR + 2 * p + 1] = (R)(re * t.shape_m[p] - t.wrd[p]);
            }
        }
    }
}

// store d[] and, on wall rows, the FP64 partial of what leaves next step
template <Storage S, int V, bool SRND>
__device__ __forceinline__ void scatter2d(typename St<S>::T *__restrict__ dst,
                                          double *__restrict__ a_next,
                                          const PairTable<typename St<S>::R> &t,
                                          const StepScalars<typename St<S>::R> &s, int64_t n, int i,
                                          int j, const typename St<S>::R (&d)[V], uint32_t step) {
    using T = typename St<S>::T;
    constexpr int NR = V & 1, NP = V / 2;
    const int nx = s.nx, ny = s.ny, H = s.halo;
    const int64_t plane = s.plane;
    uint32_t key = 0;
    if constexpr (S == Storage::F16DEV && SRND) key = node_key(n, step);
    T v[V];
    if constexpr (NR) v[0] = encode_dev<S, SRND>(d[0], t.wr00, t.inv_wr00, key >> 19);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        uint32_t r = 0;
        if constexpr (S == Storage::F16DEV && SRND) r = pcg_hash(key + (uint32_t)p);
        v[NR + 2 * p] = encode_dev<S, SRND>(d[NR + 2 * p], t.wr0[p], t.inv_wr0[p], r);
        v[NR + 2 * p + 1] = encode_dev<S, SRND>(d[NR + 2 * p + 1], t.wr0[p], t.inv_wr0[p], r >> 16);
    }
#pragma unroll
    for (int a = 0; a < V; ++a) dst[(int64_t)a * plane + n] = v[a];
    if (j < H || j >= ny - H) {
        double lo = 0.0, hi = 0.0;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int ey = t.ey[p];
            const double vp = stored_value<S>(v[NR + 2 * p], t.wrd[p]);
            const double vm = stored_value<S>(v[NR + 2 * p + 1], t.wrd[p]);
            if (j + ey < 0) lo += vp;
            if (j - ey < 0) lo += vm;
            if (j + ey >= ny) hi += vp;
            if (j - ey >= ny) hi += vm;
        }
        if (j < H) a_next[(int64_t)j * nx + i] = lo;
        if (j >= ny - H) a_next[(int64_t)(H + (ny - 1 - j)) * nx + i] = hi;
    }
}

template <int V, int NH, Storage S>
__global__ __launch_bounds__(256) void k_step2d(StepBuffers b, PairTable<typename St<S>::R> t,
                                                StepScalars<typename St<S>::R> s, int remap,
                                                uint32_t step) {
    using R = typename St<S>::R;
    using T = typename St<S>::T;
    int64_t blk = blockIdx.x;
    if (remap) blk = remap_block(blk, gridDim.x);
    const int64_t n = blk * blockDim.x + threadIdx.x;
    if (n >= s.nodes) return;
    const int j = (int)(n / s.nx);
    const int i = (int)(n - (int64_t)j * s.nx);
    R d[V];
    gather2d<S, V>((const T *)b.src, b.a_cur, t, s, i, j, d);
    Collide2D<R, V, NH>::relax(d, t, s);
    scatter2d<S, V, true>((T *)b.dst, b.a_next, t, s, n, i, j, d, step);
}

// ---------------------------------------------------------------------------
// observation: moments of the streamed state, FP64 partial sums per block
// ---------------------------------------------------------------------------
__device__ __forceinline__ void block_sum2(double a, double b, double *partial) {
    __shared__ double sa[16], sb[16];
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        sa[wv] = a;
        sb[wv] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0.0, tb = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            ta += sa[w];
            tb += sb[w];
        }
        partial[2 * blockIdx.x] = ta;
        partial[2 * blockIdx.x + 1] = tb;
    }
}

template <int V, int NH, Storage S>
__global__ __launch_bounds__(256) void k_observe2d(const void *src, const double *a_cur,
                                                   double *rho_out, double *u_out, double *partial,
                                                   PairTable<typename St<S>::R> t,
                                                   StepScalars<typename St<S>::R> s) {
    using R = typename St<S>::R;
    using T = typename St<S>::T;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double ux_d = 0.0, rho_d = 0.0;
    if (n < s.nodes) {
        const int j = (int)(n / s.nx);
        const int i = (int)(n - (int64_t)j * s.nx);
        R d[V];
        gather2d<S, V>((const T *)src, a_cur, t, s, i, j, d);
        R drho, rho, ux, uy, sxx, sxy, syy;
        Collide2D<R, V, NH>::moments(d, t, s, drho, rho, ux, uy, sxx, sxy, syy);
        rho_d = (double)s.rho0d + (double)drho;
        ux_d = (double)ux;
        if (rho_out) rho_out[n] = rho_d;
        if (u_out) {
            u_out[3 * n] = (double)ux;
            u_out[3 * n + 1] = (double)uy;
            u_out[3 * n + 2] = 0.0;
        }
    }
    block_sum2(ux_d, rho_d, partial);
}

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

// ---------------------------------------------------------------------------
// init / import / export
// ---------------------------------------------------------------------------
template <typename R, int V, int NH>
__device__ __forceinline__ void equilibrium_dev(const PairTable<R> &t, const StepScalars<R> &s,
                                                double rho_d, R ux, R uy, R uz, R (&d)[V]) {
    // f^(0) - w rho0 = w [ (rho - rho0) + rho sum_{n>=1} P_n / n! ]
    constexpr int NR = V & 1, NP = V / 2;
    const R drho = (R)(rho_d - (double)s.rho0d);
    const R rho = (R)rho_d;
    const R u2 = ux * ux + uy * uy + uz * uz;
    if constexpr (NR) d[0] = t.w0 * (drho + rho * (s.cn[2] * (-u2) + s.cn[4] * R(3) * u2 * u2));
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const R ue = ux * t.xi[p][0] + uy * t.xi[p][1] + uz * t.xi[p][2];
        R Pm = 1, P = ue, even = 0, odd = ue;
        for (int k = 1; k < NH; ++k) {
            const R Pn = ue * P - R(k) * u2 * Pm;
            Pm = P;
            P = Pn;
            if ((k + 1) & 1)
                odd += s.cn[k + 1] * P;
            else
                even += s.cn[k + 1] * P;
        }
        d[NR + 2 * p] = t.w[p] * (drho + rho * (even + odd));
        d[NR + 2 * p + 1] = t.w[p] * (drho + rho * (even - odd));
    }
}

template <int V, int NH, Storage S>
__global__ __launch_bounds__(256) void k_init2d(void *dst, double *a_out, const double *rho_in,
                                                const double *u_in,
                                                PairTable<typename St<S>::R> t,
                                                StepScalars<typename St<S>::R> s, uint32_t step) {
    using R = typename St<S>::R;
    using T = typename St<S>::T;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= s.nodes) return;
    const int j = (int)(n / s.nx);
    const int i = (int)(n - (int64_t)j * s.nx);
    const double rho = rho_in ? rho_in[n] : s.rho0d;
    R ux = 0, uy = 0;
    if (u_in) {
        ux = (R)u_in[3 * n];
        uy = (R)u_in[3 * n + 1];
    }
    R d[V];
    equilibrium_dev<R, V, NH>(t, s, rho, ux, uy, R(0), d);
    scatter2d<S, V, false>((T *)dst, a_out, t, s, n, i, j, d, step);
}

template <int V, int NH, Storage S>
__global__ __launch_bounds__(256) void k_import2d(void *dst, double *a_out, const double *in,
                                                  PairTable<typename St<S>::R> t,
                                                  StepScalars<typename St<S>::R> s, uint32_t step) {
    using R = typename St<S>::R;
    using T = typename St<S>::T;
    constexpr int NR = V & 1, NP = V / 2;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= s.nodes) return;
    const int j = (int)(n / s.nx);
    const int i = (int)(n - (int64_t)j * s.nx);
    R d[V];
    if constexpr (NR) d[0] = (R)(in[n] - t.wrd0);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        d[NR + 2 * p] = (R)(in[(int64_t)(NR + 2 * p) * s.nodes + n] - t.wrd[p]);
        d[NR + 2 * p + 1] = (R)(in[(int64_t)(NR + 2 * p + 1) * s.nodes + n] - t.wrd[p]);
    }
    scatter2d<S, V, false>((T *)dst, a_out, t, s, n, i, j, d, step);
}

template <int V, int NH, Storage S>
__global__ __launch_bounds__(256) void k_export(const void *src, double *out,
                                                PairTable<typename St<S>::R> t,
                                                StepScalars<typename St<S>::R> s) {
    using T = typename St<S>::T;
    constexpr int NR = V & 1, NP = V / 2;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= s.nodes) return;
    const T *f = (const T *)src;
    if constexpr (NR) out[n] = stored_value<S>(f[n], t.wrd0);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        for (int m = 0; m < 2; ++m) {
            const int a = NR + 2 * p + m;
            out[(int64_t)a * s.nodes + n] = stored_value<S>(f[(int64_t)a * s.plane + n], t.wrd[p]);
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int hip_ok(hipError_t e, const char *what) {
    if (e != hipSuccess) return fail(LBM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return LBM_OK;
}

static inline unsigned blocks_for(int64_t nodes) { return (unsigned)((nodes + 255) / 256); }

int observe_blocks(int64_t nodes) { return (int)blocks_for(nodes); }

template <int V, int NH, Storage S>
struct L2 {
    using R = typename St<S>::R;
    static int step(const StepBuffers &b, const void *tab, const void *sc, hipStream_t st,
                    int remap, uint32_t stp) {
        const auto &t = *(const PairTable<R> *)tab;
        const auto &s = *(const StepScalars<R> *)sc;
        hipLaunchKernelGGL((k_step2d<V, NH, S>), dim3(blocks_for(s.nodes)), dim3(256), 0, st, b, t,
                           s, remap, stp);
        return hip_ok(hipGetLastError(), "step kernel launch");
    }
    static int init(void *dst, double *a_out, const double *rho, const double *u, const void *tab,
                    const void *sc, hipStream_t st, uint32_t stp) {
        const auto &t = *(const PairTable<R> *)tab;
        const auto &s = *(const StepScalars<R> *)sc;
        hipLaunchKernelGGL((k_init2d<V, NH, S>), dim3(blocks_for(s.nodes)), dim3(256), 0, st, dst,
                           a_out, rho, u, t, s, stp);
        return hip_ok(hipGetLastError(), "init kernel launch");
    }
    static int observe(const void *src, const double *a_cur, double *rho, double *u,
                       double *partial, const void *tab, const void *sc, hipStream_t st) {
        const auto &t = *(const PairTable<R> *)tab;
        const auto &s = *(const StepScalars<R> *)sc;
        hipLaunchKernelGGL((k_observe2d<V, NH, S>), dim3(blocks_for(s.nodes)), dim3(256), 0, st,
                           src, a_cur, rho, u, partial, t, s);
        return hip_ok(hipGetLastError(), "observe kernel launch");
    }
    static int exportp(const void *src, double *out, const void *tab, const void *sc,
                       hipStream_t st) {
        const auto &t = *(const PairTable<R> *)tab;
        const auto &s = *(const StepScalars<R> *)sc;
        hipLaunchKernelGGL((k_export<V, NH, S>), dim3(blocks_for(s.nodes)), dim3(256), 0, st, src,
                           out, t, s);
        return hip_ok(hipGetLastError(), "export kernel launch");
    }
    static int importp(void *dst, double *a_out, const double *in, const void *tab, const void *sc,
                       hipStream_t st, uint32_t stp) {
        const auto &t = *(const PairTable<R> *)tab;
        const auto &s = *(const StepScalars<R> *)sc;
        hipLaunchKernelGGL((k_import2d<V, NH, S>), dim3(blocks_for(s.nodes)), dim3(256), 0, st,
                           dst, a_out, in, t, s, stp);
        return hip_ok(hipGetLastError(), "import kernel launch");
    }
    static constexpr Launch table{&step, &init, &observe, &exportp, &importp};
};

int launch_finalize(const double *partials, int n, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, partials, n, out);
    return hip_ok(hipGetLastError(), "finalize kernel launch");
}

struct Entry {
    int dim, V, N;
    Storage s;
    const Launch *l;
};

#define LBM_2D(V, N)                                                        \
    {2, V, N, Storage::F64, &L2<V, N, Storage::F64>::table},                \
        {2, V, N, Storage::F32, &L2<V, N, Storage::F32>::table},            \
        {2, V, N, Storage::F32RAW, &L2<V, N, Storage::F32RAW>::table},      \
        {2, V, N, Storage::F16DEV, &L2<V, N, Storage::F16DEV>::table}

static const Entry kEntries[] = {
    LBM_2D(17, 3), LBM_2D(37, 4), LBM_2D(37, 3), LBM_2D(16, 3), LBM_2D(33, 4), LBM_2D(32, 3),
};

const Launch *find_launch(int dim, int V, int N, Storage s) {
    for (const auto &e : kEntries)
        if (e.dim == dim && e.V == V && e.N == N && e.s == s) return e.l;
    return nullptr;
}

}  // namespace lbm
