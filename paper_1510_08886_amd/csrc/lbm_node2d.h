// Per-node arithmetic of the 2D channel update, shared by the HBM step kernel
// and the LDS-resident batched kernel so both compute bit-identical values:
// moments, equilibrium + force + BGK relaxation of the modified populations,
// wall-slot completion and the FP64 wall-flux partials.
#pragma once

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
// wall slots and wall-flux partials (2D channel)
// ---------------------------------------------------------------------------
// raw[] holds the stored values at the (clamped) pull sources; decode them to
// deviations and replace the values whose source lies outside the channel by
// the diffuse-wall populations. a_cur holds the FP64 partials of the column
// as [face][row < HN][column] with column stride nx.
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

// FP64 partial, per wall row and column, of the just-stored populations that
// leave through each face in the next streaming step (plus the constant
// w rho0 parts for deviation storages).
template <class SET, Storage S>
__device__ __forceinline__ void wall_partials2d(const typename St<S>::T (&v)[SET::V],
                                                const PairTable<typename St<S>::R> &t,
                                                const StepScalars<typename St<S>::R> &s, int i,
                                                int j, double *__restrict__ a_next) {
    constexpr int NR = SET::NR, HN = SET::HN;
    const int nx = s.nx, ny = s.ny;
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

}  // namespace lbm
