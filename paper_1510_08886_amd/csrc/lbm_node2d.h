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

// Equilibrium + force + BGK relaxation per velocity pair (e, -e), with the
// Hermite sums regrouped as polynomials in the integer velocity e, whose
// coefficients are formed once per node (ue = u.xi, u2 = |u|^2, xi = c e):
//   f^(0)/w  = drho + rho [1 + ue + (ue^2 - u2)/2 + (ue^3 - 3 u2 ue)/6
//                          + (ue^4 - 6 u2 ue^2 + 3 u2^2)/24
//                          + (ue^5 - 10 u2 ue^3 + 15 u2^2 ue)/120]   (terms up to N)
//   tau F/w  = tau rho [(g.xi) + (g.xi)(u.xi) - g.u]
//              + tau/2 (g.xi)(a2 : xi xi - tr a2) - tau (a2 g).xi  (Eq. nm.4)
// so that, with g along x,
//   even(e) = C0 + ue^2 (C2 + C4 ue^2) + e_x T ue
//   odd(e)  = ue (R1 + ue^2 (R3 + rc5 ue^2)) + e.L + e_x (e_x^2 Kxx + e_y^2 Kyy + e_x e_y Kxy)
// and fbar* = fbar + omega (w (even +- odd) - fbar) (Eq. nm.8) on deviations.
// N5 compiles the fifth-order term (Hermite order 5, sets of quadrature order
// 9); without it rc5 = 0 and odd = ue (R1 + rc3 ue^2).
template <class SET, typename R, bool N5 = false>
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
    const R gxc = gx * c;
    const R uxc = ux * c, uyc = uy * c;
    const R u2 = ux * ux + uy * uy;
    const R tr = s.tau * rho;
    const R rc2 = rho * s.cn[2], rc3 = rho * s.cn[3], rc4 = rho * s.cn[4];
    const R om = s.omega;
    // even part: C0 is also the rest velocity's value (ue = 0)
    const R C0 = fma(R(3) * rc4 * u2, u2, fma(-rc2, u2, drho - tr * ux * gx));
    const R C2 = fma(R(-6) * rc4, u2, rc2);
    const R C4 = rc4;
    const R T = tr * gxc;
    // odd part
    const R rc5 = N5 ? rho * s.cn[5] : R(0);
    const R R1 = N5 ? fma(R(15) * rc5 * u2, u2, fma(R(-3) * rc3, u2, rho)) : fma(R(-3) * rc3, u2, rho);
    const R R3 = N5 ? fma(R(-10) * rc5, u2, rc3) : rc3;
    const R hgt = R(0.5) * s.tau * gxc;
    const R Lx = fma(gxc, fma(R(-0.5) * s.tau, tra2, tr), -s.tau * a2xx * gxc);
    const R Ly = -s.tau * a2xy * gxc;
    const R Kxx = hgt * a2xx * c2, Kyy = hgt * a2yy * c2, Kxy = R(2) * hgt * a2xy * c2;
    if constexpr (NR) d[0] = fma(om, fma(t.w0, C0, -d[0]), d[0]);
    for_pairs<SET::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int ex = SET::EX[p], ey = SET::EY[p];
        const R ue = lin2<ex, ey>(uxc, uyc);
        const R ue2 = ue * ue;
        R even = fma(fma(C4, ue2, C2), ue2, C0);
        if constexpr (ex != 0) even = fma(mulk<ex>(T), ue, even);
        R f = lin2<ex, ey>(Lx, Ly);
        f = addk<ex * ex * ex>(f, Kxx);
        f = addk<ex * ey * ey>(f, Kyy);
        f = addk<ex * ex * ey>(f, Kxy);
        R odd;
        if constexpr (N5)
            odd = fma(ue, fma(ue2, fma(rc5, ue2, R3), R1), f);
        else
            odd = fma(ue, fma(R3, ue2, R1), f);
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
// Slot of the velocity (e_x, -e_y) for slot a (reflection at a wall normal to
// y); the velocity sets are symmetric under it.
template <class SET>
constexpr int mirror_slot(int a) {
    constexpr int NR = SET::NR;
    if (NR && a == 0) return 0;
    const int p = (a - NR) / 2;
    const int sg = (a - NR) % 2 ? -1 : 1;
    const int ex = sg * SET::EX[p], ey = -sg * SET::EY[p];
    for (int q = 0; q < SET::NP; ++q) {
        if (SET::EX[q] == ex && SET::EY[q] == ey) return NR + 2 * q;
        if (SET::EX[q] == -ex && SET::EY[q] == -ey) return NR + 2 * q + 1;
    }
    return -1;
}
template <class SET>
constexpr bool mirror_complete() {
    for (int a = 0; a < SET::V; ++a)
        if (mirror_slot<SET>(a) < 0) return false;
    return true;
}

// No specular partners (fully diffuse walls).
template <typename T>
struct NoMirror {
    __device__ __forceinline__ T operator()(int, int, int) const { return T(0); }
};

// raw[] holds the stored values at the (clamped) pull sources; decode them to
// deviations and replace the values whose source lies outside the channel by
// the wall's populations. a_col points at the FP64 partials of the node's
// column, [face][row < HN] with row stride `stride` (the global partials
// [face][row][column] have stride nx).
//
// Maxwell's wall with accommodation alpha (s.specular when alpha < 1; the
// paper treats alpha = 1): a fraction alpha of the populations that reach an
// element is re-emitted diffusely, alpha rho_eff w (1 - dt/2 g.xi), and the
// rest reflected specularly: the unknown slot (e_x, e_y) of node (i, j) whose
// source row j - e_y lies beyond a wall receives 1 - alpha times the
// post-collision population (e_x, -e_y) of the node (i - e_x, jm) mirrored
// about that wall, jm = -1 - (j - e_y) below and 2 ny - 1 - (j - e_y) above
// (the straight path from x - e folded at the wall plane). mir(slot, jm, e_x)
// returns that stored value for the unknown slot `slot` (y-reflected velocity
// mirror_slot(slot)); it is only called when s.specular.
template <class SET, Storage S, class MIR = NoMirror<typename St<S>::T>>
__device__ __forceinline__ void complete2d_col(const typename St<S>::T (&raw)[SET::V],
                                               const double *__restrict__ a_col, int stride,
                                               const PairTable<typename St<S>::R> &t,
                                               const StepScalars<typename St<S>::R> &s, int j,
                                               typename St<S>::R (&d)[SET::V],
                                               const MIR &mir = MIR()) {
    using T = typename St<S>::T;
    using R = typename St<S>::R;
    constexpr int NR = SET::NR, HN = SET::HN;
    const int ny = s.ny;
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
            alo += a_col[r * stride];
            ahi += a_col[(HN + r) * stride];
        }
        const double rlo = alo * s.invD[0], rhi = ahi * s.invD[1];
        static_assert(mirror_complete<SET>(), "velocity set closed under y reflection");
        // wall population w (rho_eff (1 - dt/2 g.xi)) as a deviation from w rho0
        const double rho0 = s.rho0d, hgc = s.hgc;
        for_pairs<SET::NP>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            constexpr int ex = SET::EX[p], ey = SET::EY[p];
            if constexpr (ey != 0) {
                const double wd = (double)t.w[p];
                constexpr int mp = mirror_slot<SET>(NR + 2 * p), mm = mirror_slot<SET>(NR + 2 * p + 1);
                int js = j - ey;
                if (js < 0 || js >= ny) {
                    const double re = js < 0 ? rlo : rhi;
                    double dv = wd * (re * (1.0 - hgc * ex) - rho0);
                    if (s.specular) {
                        const int jm = js < 0 ? -1 - js : 2 * ny - 1 - js;
                        const R sp = decode_dev<S>((T)mir(NR + 2 * p, jm, ex),
                                                   t.wr0[(mp - NR) / 2]);
                        dv = s.alpha * dv + (1.0 - s.alpha) * (double)sp;
                    }
                    d[NR + 2 * p] = (R)dv;
                }
                js = j + ey;
                if (js < 0 || js >= ny) {
                    const double re = js < 0 ? rlo : rhi;
                    double dv = wd * (re * (1.0 + hgc * ex) - rho0);
                    if (s.specular) {
                        const int jm = js < 0 ? -1 - js : 2 * ny - 1 - js;
                        const R sp = decode_dev<S>((T)mir(NR + 2 * p + 1, jm, -ex),
                                                   t.wr0[(mm - NR) / 2]);
                        dv = s.alpha * dv + (1.0 - s.alpha) * (double)sp;
                    }
                    d[NR + 2 * p + 1] = (R)dv;
                }
            }
        });
    }
}

template <class SET, Storage S, class MIR = NoMirror<typename St<S>::T>>
__device__ __forceinline__ void complete2d(const typename St<S>::T (&raw)[SET::V],
                                           const double *__restrict__ a_cur,
                                           const PairTable<typename St<S>::R> &t,
                                           const StepScalars<typename St<S>::R> &s, int i, int j,
                                           typename St<S>::R (&d)[SET::V], const MIR &mir = MIR()) {
    complete2d_col<SET, S>(raw, a_cur + i, s.nx, t, s, j, d, mir);
}

// Specular partner in a kDirect AoSoA-64 population array (node n at
// aos_base(n), velocity alpha in slot alpha) that the step does not write:
// specular walls are stepped ping-pong only, since in the in-place layouts the
// mirrored node overwrites that population in the same step.
template <class SET, typename T>
struct ArrayMirror {
    const T *A;
    int i, nx;
    __device__ __forceinline__ T operator()(int slot, int jm, int ex) const {
        const int col = wrap_col(i - ex, nx, SET::H);
        const int at = mirror_slot<SET>(slot);
        return A[aos_base<SET::V>((uint32_t)jm * (uint32_t)nx + (uint32_t)col) + 64u * (uint32_t)at];
    }
};

// FP64 partial, per wall row and column, of the just-stored populations that
// leave through each face in the next streaming step (plus the constant
// w rho0 parts for deviation storages), into the column's partials a_col
// ([face][row < HN], row stride `stride`).
template <class SET, Storage S>
__device__ __forceinline__ void wall_partials2d_col(const typename St<S>::T (&v)[SET::V],
                                                    const PairTable<typename St<S>::R> &t,
                                                    const StepScalars<typename St<S>::R> &s,
                                                    int j, double *__restrict__ a_col,
                                                    int stride) {
    constexpr int NR = SET::NR, HN = SET::HN;
    const int ny = s.ny;
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
        if (j < HN) a_col[j * stride] = s.kA[0][j] + lo;
        if (j >= ny - HN) a_col[(HN + (ny - 1 - j)) * stride] = s.kA[1][ny - 1 - j] + hi;
    }
}

template <class SET, Storage S>
__device__ __forceinline__ void wall_partials2d(const typename St<S>::T (&v)[SET::V],
                                                const PairTable<typename St<S>::R> &t,
                                                const StepScalars<typename St<S>::R> &s, int i,
                                                int j, double *__restrict__ a_next) {
    wall_partials2d_col<SET, S>(v, t, s, j, a_next + i, s.nx);
}

}  // namespace lbm
