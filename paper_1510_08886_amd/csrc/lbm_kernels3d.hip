// HIP kernels for gfx950: the fused pull-stream + diffuse Maxwell wall + BGK
// update (Eq. nm.8) of a 3D duct: x periodic, walls normal to y and z.
//
// Node n = (k * ny + j) * nx + i; populations in 64-node blocks (aos_base), one
// array updated in place (PopLayout). Neighbour accesses are clamped into the
// duct in y and z so every access is valid; the populations whose source lies
// outside are replaced by the diffuse-wall populations rho_eff w (1 - dt/2
// g.xi) of Eqs. nm.14 / nm.15.
//
// Wall elements: an unknown slot (x, alpha), whose virtual source x - e_alpha
// lies outside, and the absorbed population (x, -alpha) cross the same
// segment; both belong to the wall cell of the fluid node x on the face the
// segment crosses first going outward (ties to the y face). y faces have
// elements (k, i), z faces (j, i). rho_eff(e) = A(e) / D(e): A(e) is the FP64
// sum of the post-collision populations that left through e, kept per wall
// row (distance of the node from the face) and summed by the consumer; D(e)
// depends only on the element's position along the face (k or j) and is
// tabulated on the host, since slots near the duct's edges may belong to the
// other face.
#include <hip/hip_runtime.h>

#include <utility>

#include "lbm_device.h"

namespace lbm {

enum : int { kYLo = 0, kYHi = 1, kZLo = 2, kZHi = 3 };

template <typename R>
struct Moments3D {
    R drho, rho, ux, uy, uz, sxx, syy, szz, sxy, sxz, syz;
};

template <class SET, typename R>
__device__ __forceinline__ Moments3D<R> moments3d(const R (&d)[SET::V], const StepScalars<R> &s,
                                                  R c) {
    constexpr int NR = SET::NR;
    R drho = NR ? d[0] : R(0);
    R jx = 0, jy = 0, jz = 0, sxx = 0, syy = 0, szz = 0, sxy = 0, sxz = 0, syz = 0;
    for_pairs<SET::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int ex = SET::EX[p], ey = SET::EY[p], ez = SET::EZ[p];
        const R dp = d[NR + 2 * p], dm = d[NR + 2 * p + 1];
        const R sum = dp + dm, dif = dp - dm;
        drho += sum;
        jx = addk<ex>(jx, dif);
        jy = addk<ey>(jy, dif);
        jz = addk<ez>(jz, dif);
        sxx = addk<ex * ex>(sxx, sum);
        syy = addk<ey * ey>(syy, sum);
        szz = addk<ez * ez>(szz, sum);
        sxy = addk<ex * ey>(sxy, sum);
        sxz = addk<ex * ez>(sxz, sum);
        syz = addk<ey * ez>(syz, sum);
    });
    Moments3D<R> m;
    const R c2 = c * c;
    m.drho = drho;
    m.rho = s.rho0 + drho;
    const R inv = R(1) / m.rho;
    m.ux = fma(s.half_dt_g[0], m.rho, jx * c) * inv;
    m.uy = jy * c * inv;
    m.uz = jz * c * inv;
    m.sxx = sxx * c2;
    m.syy = syy * c2;
    m.szz = szz * c2;
    m.sxy = sxy * c2;
    m.sxz = sxz * c2;
    m.syz = syz * c2;
    return m;
}

// Equilibrium + force (Eq. nm.4, g along x) + BGK relaxation per velocity pair,
// with the Hermite sums as polynomials in the integer velocity e whose
// coefficients are formed once per node (as in the 2D channel):
//   even(e) = C0 + ue^2 (C2 + C4 ue^2) + e_x T ue
//   odd(e)  = ue (R1 + rc3 ue^2) + e.L
//             + e_x (e_x^2 Kxx + e_y^2 Kyy + e_z^2 Kzz + e_x e_y Kxy + e_x e_z Kxz + e_y e_z Kyz)
template <class SET, typename R>
__device__ __forceinline__ void relax3d(R (&d)[SET::V], const PairTable<R> &t,
                                        const StepScalars<R> &s, R c) {
    constexpr int NR = SET::NR;
    const auto m = moments3d<SET, R>(d, s, c);
    const R drho = m.drho, rho = m.rho, ux = m.ux, uy = m.uy, uz = m.uz;
    const R gx = s.g[0];
    // a2 = Pi(f) - rho I from fbar by inverting Eq. nm.7 (deviation form)
    const R hr = s.h * rho;
    const R htr = hr * s.tau;
    const R i1h = s.inv1h;
    const R a2xx = (m.sxx - drho + hr * ux * ux + R(2) * htr * gx * ux) * i1h;
    const R a2yy = (m.syy - drho + hr * uy * uy) * i1h;
    const R a2zz = (m.szz - drho + hr * uz * uz) * i1h;
    const R a2xy = (m.sxy + hr * ux * uy + htr * gx * uy) * i1h;
    const R a2xz = (m.sxz + hr * ux * uz + htr * gx * uz) * i1h;
    const R a2yz = (m.syz + hr * uy * uz) * i1h;
    const R tra2 = a2xx + a2yy + a2zz;
    const R c2 = c * c;
    const R gxc = gx * c;
    const R uxc = ux * c, uyc = uy * c, uzc = uz * c;
    const R u2 = ux * ux + uy * uy + uz * uz;
    const R tr = s.tau * rho;
    const R rc2 = rho * s.cn[2], rc3 = rho * s.cn[3], rc4 = rho * s.cn[4];
    const R om = s.omega;
    const R C0 = fma(R(3) * rc4 * u2, u2, fma(-rc2, u2, drho - tr * ux * gx));
    const R C2 = fma(R(-6) * rc4, u2, rc2);
    const R C4 = rc4;
    const R T = tr * gxc;
    const R R1 = fma(R(-3) * rc3, u2, rho);
    const R hgt = R(0.5) * s.tau * gxc;
    const R Lx = fma(gxc, fma(R(-0.5) * s.tau, tra2, tr), -s.tau * a2xx * gxc);
    const R Ly = -s.tau * a2xy * gxc;
    const R Lz = -s.tau * a2xz * gxc;
    const R hc2 = hgt * c2;
    const R Kxx = hc2 * a2xx, Kyy = hc2 * a2yy, Kzz = hc2 * a2zz;
    const R Kxy = R(2) * hc2 * a2xy, Kxz = R(2) * hc2 * a2xz, Kyz = R(2) * hc2 * a2yz;
    if constexpr (NR) d[0] = fma(om, fma(t.w0, C0, -d[0]), d[0]);
    for_pairs<SET::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int ex = SET::EX[p], ey = SET::EY[p], ez = SET::EZ[p];
        const R ue = lin3<ex, ey, ez>(uxc, uyc, uzc);
        const R ue2 = ue * ue;
        R even = fma(fma(C4, ue2, C2), ue2, C0);
        if constexpr (ex != 0) even = fma(mulk<ex>(T), ue, even);
        R f = lin3<ex, ey, ez>(Lx, Ly, Lz);
        f = addk<ex * ex * ex>(f, Kxx);
        f = addk<ex * ey * ey>(f, Kyy);
        f = addk<ex * ez * ez>(f, Kzz);
        f = addk<ex * ex * ey>(f, Kxy);
        f = addk<ex * ex * ez>(f, Kxz);
        f = addk<ex * ey * ez>(f, Kyz);
        const R odd = fma(ue, fma(rc3, ue2, R1), f);
        const R w = t.w[p];
        R &dp = d[NR + 2 * p];
        R &dm = d[NR + 2 * p + 1];
        dp = fma(om, fma(w, even + odd, -dp), dp);
        dm = fma(om, fma(w, even - odd, -dm), dm);
    });
}

// fraction of the step at which a particle at coordinate `from`, moving with
// integer velocity component v != 0, crosses the wall plane ahead of it
__device__ __forceinline__ double exit_time(int from, int v, int n) {
    const double plane = v > 0 ? (double)n - 0.5 : -0.5;
    return (plane - (double)from) / (double)v;
}

// face of the segment from node (j, k) along (vy, vz) to a point outside in y
// (oy) and/or z (oz): the first one crossed, ties to y
__device__ __forceinline__ int first_face(int j, int k, int vy, int vz, bool oy, bool oz, int ny,
                                          int nz) {
    bool use_z = oz;
    if (oy && oz) use_z = exit_time(k, vz, nz) < exit_time(j, vy, ny);
    if (use_z) return vz < 0 ? kZLo : kZHi;
    return vy < 0 ? kYLo : kYHi;
}

// ---------------------------------------------------------------------------
// neighbour addressing of the in-place array (PopLayout): position of slot 0
// of node (k - dz, j - dy, i - dx), |dz|, |dy| <= HN, |dx| <= H, rows clamped
// into the duct (every address valid), x periodic; ALIGNED: a row part
// (uniform when the row is) plus a column part
// ---------------------------------------------------------------------------
template <class SET, bool ALIGNED>
struct Nbr3 {
    static constexpr int H = SET::H, HN = SET::HN, V = SET::V;
    int ry[2 * HN + 1], rz[2 * HN + 1];
    uint32_t col[2 * H + 1];
    uint32_t rowstride;
    int nx, ny;
    template <class SC>
    __device__ __forceinline__ Nbr3(const SC &s, int i, int j, int k) : nx(s.nx), ny(s.ny) {
        rowstride = (uint32_t)s.nx * V;
#pragma unroll
        for (int q = -HN; q <= HN; ++q) {
            ry[q + HN] = min(max(j - q, 0), s.ny - 1);
            rz[q + HN] = min(max(k - q, 0), s.nz - 1);
        }
#pragma unroll
        for (int q = -H; q <= H; ++q) {
            const uint32_t x = (uint32_t)wrap_col(i - q, s.nx, H);
            col[q + H] = ALIGNED ? (x >> 6) * (uint32_t)(64 * V) + (x & 63u) : x;
        }
    }
    __device__ __forceinline__ Ix at(int dz, int dy, int dx) const {
        const uint32_t row = (uint32_t)rz[dz + HN] * (uint32_t)ny + (uint32_t)ry[dy + HN];
        if constexpr (ALIGNED)
            return {col[dx + H], row * rowstride, 0u};
        else
            return {aos_base<V>(row * (uint32_t)nx + col[dx + H]), 0u, 0u};
    }
};

// pull of the pre-collision values: population +e_p of x from x - e_p, in
// slot -e_p (SWAP, kLocal) or +e_p (kDirect)
template <class SET, bool SWAP, class NB, class P, typename T>
__device__ __forceinline__ void read_pull3(const P &pop, const NB &nb, Ix own, T (&raw)[SET::V]) {
    constexpr int NR = SET::NR;
    if constexpr (NR) raw[0] = pop.ld(own);
    for_pairs<SET::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int ex = SET::EX[p], ey = SET::EY[p], ez = SET::EZ[p];
        raw[NR + 2 * p] = pop.ld(slot_of(nb.at(ez, ey, ex), SWAP ? NR + 2 * p + 1 : NR + 2 * p));
        raw[NR + 2 * p + 1] =
            pop.ld(slot_of(nb.at(-ez, -ey, -ex), SWAP ? NR + 2 * p : NR + 2 * p + 1));
    });
}

// home of post-collision population +e_p (PLUS) or -e_p of node x in the
// kStreamed layout: slot +-e_p of x +- e_p, or the node's own slot of the
// opposite velocity when x +- e_p lies outside the duct. INTERIOR: the node
// is at least HN rows from every wall (every destination inside).
template <class SET, int p, bool PLUS, bool INTERIOR, class P, class NB>
__device__ __forceinline__ Ix home3d(const NB &nb, Ix own, int j, int k, int ny, int nz) {
    constexpr int NR = SET::NR;
    constexpr int sx = PLUS ? SET::EX[p] : -SET::EX[p];
    constexpr int sy = PLUS ? SET::EY[p] : -SET::EY[p];
    constexpr int sz = PLUS ? SET::EZ[p] : -SET::EZ[p];
    constexpr int slot = PLUS ? NR + 2 * p : NR + 2 * p + 1, opp = PLUS ? NR + 2 * p + 1 : NR + 2 * p;
    if constexpr ((sy == 0 && sz == 0) || INTERIOR) {
        return slot_of(nb.at(-sz, -sy, -sx), slot);
    } else {
        bool inside = true;
        if constexpr (sy != 0) inside = inside && (unsigned)(j + sy) < (unsigned)ny;
        if constexpr (sz != 0) inside = inside && (unsigned)(k + sz) < (unsigned)nz;
        const Ix there = slot_of(nb.at(-sz, -sy, -sx), slot), here = slot_of(own, opp);
        return inside ? P::flat(there) : P::flat(here);
    }
}

// post-collision values -> kStreamed layout
template <class SET, bool STREAM, bool INTERIOR, class NB, class P, typename T>
__device__ __forceinline__ void write_gs3(const P &pop, const NB &nb, Ix own, int j, int k, int ny,
                                          int nz, const T (&v)[SET::V]) {
    constexpr int NR = SET::NR;
    if constexpr (NR) pop.template st<STREAM>(own, v[0]);
    for_pairs<SET::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        pop.template st<STREAM>(home3d<SET, p, true, INTERIOR, P>(nb, own, j, k, ny, nz),
                                v[NR + 2 * p]);
        pop.template st<STREAM>(home3d<SET, p, false, INTERIOR, P>(nb, own, j, k, ny, nz),
                                v[NR + 2 * p + 1]);
    });
}

template <class SET, Storage S>
__device__ __forceinline__ void complete3d(const typename St<S>::T (&raw)[SET::V],
                                           const double *__restrict__ a_cur,
                                           const double *__restrict__ invd,
                                           const PairTable<typename St<S>::R> &t,
                                           const StepScalars<typename St<S>::R> &s, int i, int j,
                                           int k, typename St<S>::R (&d)[SET::V]) {
    using R = typename St<S>::R;
    constexpr int NR = SET::NR, HN = SET::HN;
    const int nx = s.nx, ny = s.ny, nz = s.nz;
    if constexpr (NR) d[0] = decode_dev<S>(raw[0], t.wr00);
    for_pairs<SET::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        d[NR + 2 * p] = decode_dev<S>(raw[NR + 2 * p], t.wr0[p]);
        d[NR + 2 * p + 1] = decode_dev<S>(raw[NR + 2 * p + 1], t.wr0[p]);
    });
    const bool ylo = j < HN, yhi = j >= ny - HN, zlo = k < HN, zhi = k >= nz - HN;
    if (!(ylo || yhi || zlo || zhi)) return;
    // rho_eff of this node's element on each face it is next to
    const int64_t fs = (int64_t)HN * max(nz, ny) * nx;
    const int64_t ey_ = (int64_t)k * nx + i, ez_ = (int64_t)j * nx + i;
    const int64_t dstride = max(nz, ny);
    double reff[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const bool near = f == kYLo ? ylo : f == kYHi ? yhi : f == kZLo ? zlo : zhi;
        if (!near) continue;
        const int64_t el = f < 2 ? ey_ : ez_;
        const int64_t epl = f < 2 ? (int64_t)nz * nx : (int64_t)ny * nx;
        double a = 0.0;
        for (int r = 0; r < HN; ++r) a += a_cur[f * fs + r * epl + el];
        reff[f] = a * invd[f * dstride + (f < 2 ? k : j)];
    }
    const double rho0 = s.rho0d, hgc = s.hgc;
    for_pairs<SET::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int ex = SET::EX[p], ey = SET::EY[p], ez = SET::EZ[p];
        if constexpr (ey != 0 || ez != 0) {
            const double wd = (double)t.w[p];
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const int sy = m ? -ey : ey, sz = m ? -ez : ez, sx = m ? -ex : ex;
                const int js = j - sy, ks = k - sz;
                const bool oy = js < 0 || js >= ny, oz = ks < 0 || ks >= nz;
                if (oy || oz) {
                    const int f = first_face(j, k, -sy, -sz, oy, oz, ny, nz);
                    d[NR + 2 * p + m] = (R)(wd * (reff[f] * (1.0 - hgc * sx) - rho0));
                }
            }
        }
    });
}

template <class SET, Storage S>
__device__ __forceinline__ void wall_partials3d(const typename St<S>::T (&v)[SET::V],
                                                const PairTable<typename St<S>::R> &t,
                                                const StepScalars<typename St<S>::R> &s, int i,
                                                int j, int k, double *__restrict__ a_next) {
    constexpr int NR = SET::NR, HN = SET::HN;
    const int nx = s.nx, ny = s.ny, nz = s.nz;
    const bool ylo = j < HN, yhi = j >= ny - HN, zlo = k < HN, zhi = k >= nz - HN;
    if (!(ylo || yhi || zlo || zhi)) return;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for_pairs<SET::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int ey = SET::EY[p], ez = SET::EZ[p];
        if constexpr (ey != 0 || ez != 0) {
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const int sy = m ? -ey : ey, sz = m ? -ez : ez;
                const int jd = j + sy, kd = k + sz;
                const bool oy = jd < 0 || jd >= ny, oz = kd < 0 || kd >= nz;
                if (oy || oz) {
                    const int f = first_face(j, k, sy, sz, oy, oz, ny, nz);
                    acc[f] += stored_value<S>(v[NR + 2 * p + m], t.wrd[p]);
                }
            }
        }
    });
    const int64_t fs = (int64_t)HN * max(nz, ny) * nx;
    const int64_t epy = (int64_t)nz * nx, epz = (int64_t)ny * nx;
    if (ylo) a_next[kYLo * fs + (int64_t)j * epy + (int64_t)k * nx + i] = acc[kYLo];
    if (yhi) a_next[kYHi * fs + (int64_t)(ny - 1 - j) * epy + (int64_t)k * nx + i] = acc[kYHi];
    if (zlo) a_next[kZLo * fs + (int64_t)k * epz + (int64_t)j * nx + i] = acc[kZLo];
    if (zhi) a_next[kZHi * fs + (int64_t)(nz - 1 - k) * epz + (int64_t)j * nx + i] = acc[kZHi];
}

__device__ __forceinline__ void node_ijk(uint32_t n, int nx, int ny, int &i, int &j, int &k) {
    const uint32_t row = n / (uint32_t)nx;
    i = (int)(n - row * nx);
    k = (int)(row / (uint32_t)ny);
    j = (int)(row - (uint32_t)k * ny);
}

// step kinds (as for the channel): ping-pong pull (kDirect), and in place
// gather/scatter (kLocal -> kStreamed) and node-local (kStreamed -> kLocal)
enum StepKind3 : int { kPingPong3 = 0, kGatherScatter3 = 1, kNodeLocal3 = 2 };

// One thread per node, blocks of up to 256 threads: one block per (x tile,
// row) when nx is a multiple of 64 (ALIGNED, compiled apart), else per 256
// consecutive nodes.
template <class SET, Storage S, bool ALIGNED, bool STREAM, int KIND>
__global__ __launch_bounds__(256)
void k_step3d(StepBuffers b, PairTable<typename St<S>::R> t, StepScalars<typename St<S>::R> s,
              uint32_t step) {
    using R = typename St<S>::R;
    using T = typename St<S>::T;
    // ALIGNED: a 2D grid of (x tile, row) blocks with row = k * ny + j, so j,
    // k and every row offset are uniform (scalar registers)
    int i, j, k;
    uint32_t n;
    if constexpr (ALIGNED) {
        const uint32_t row = blockIdx.y;
        k = (int)(row / (uint32_t)s.ny);
        j = (int)(row - (uint32_t)k * (uint32_t)s.ny);
        i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
        n = row * (uint32_t)s.nx + (uint32_t)i;
    } else {
        n = blockIdx.x * 256u + threadIdx.x;
        if (n >= (uint32_t)s.nodes) return;
        node_ijk(n, s.nx, s.ny, i, j, k);
    }
    // BUF (aligned rows, 16-bit storage): raw buffer accesses with the row and
    // slot offsets in the scalar operand (arrays below 2 GiB), which removes
    // the vector address arithmetic. Measured on MI355X: 4% faster for the
    // FP16 duct step, whose arithmetic outweighs its halved traffic; 0.4-2%
    // slower for FP32 steps (the compiler then batches the stores after the
    // collision instead of interleaving them), which keep flat addresses.
    constexpr bool BUF = ALIGNED && sizeof(T) == 2;
    T *A = (T *)b.pop;
    auto pop_at = [&](void *base) {
        if constexpr (BUF)
            return BufferPop<T>(base, (uint32_t)s.nodes * (uint32_t)(SET::V * sizeof(T)));
        else
            return GlobalPop<T>{(T *)base};
    };
    const auto pop = pop_at(A);
    const Ix own = BUF ? Ix{((uint32_t)i >> 6) * (uint32_t)(64 * SET::V) + ((uint32_t)i & 63u),
                                (uint32_t)blockIdx.y * (uint32_t)s.nx * SET::V, 0u}
                       : Ix{aos_base<SET::V>(n), 0u, 0u};
    T raw[SET::V];
    // KIND == kNodeLocal3 reads only the node's own slots
    const Nbr3<SET, ALIGNED> nb(s, i, j, k);
    if constexpr (KIND == kNodeLocal3)
        read_local<SET>(pop, own, raw);
    else
        read_pull3<SET, KIND == kGatherScatter3>(pop, nb, own, raw);
    R d[SET::V];
    complete3d<SET, S>(raw, b.a_cur, b.invd, t, s, i, j, k, d);
    relax3d<SET, R>(d, t, s, t.c);
    T v[SET::V];
    encode_all<SET, S, true>(d, t, n, step, v);
    if constexpr (KIND == kGatherScatter3 && BUF) {
        // write positions equal read positions of other velocities: 2H + 1
        // column offsets stay live (rows are scalar); nodes at least HN rows
        // from every wall (a uniform test) store without the wall selects
        constexpr int HN = SET::HN;
        if (j >= HN && j < s.ny - HN && k >= HN && k < s.nz - HN)
            write_gs3<SET, STREAM, true>(pop, nb, own, j, k, s.ny, s.nz, v);
        else
            write_gs3<SET, STREAM, false>(pop, nb, own, j, k, s.ny, s.nz, v);
    } else if constexpr (KIND == kGatherScatter3) {
        // recompute the write addresses (equal to read addresses of other
        // velocities) rather than keep them live through the collision
        int iw = i, jw = j, kw = k;
        asm volatile("" : "+v"(iw), "+v"(jw), "+v"(kw));
        const Nbr3<SET, ALIGNED> nbw(s, iw, jw, kw);
        write_gs3<SET, STREAM, false>(pop, nbw, own, jw, kw, s.ny, s.nz, v);
    } else if constexpr (KIND == kNodeLocal3) {
        write_own<SET, true, STREAM>(pop, own, v);
    } else {
        write_own<SET, false, STREAM>(pop_at(b.pop_out), own, v);
    }
    wall_partials3d<SET, S>(v, t, s, i, j, k, b.a_next);
}

template <class SET, Storage S>
__global__ __launch_bounds__(256) void k_observe3d(const void *pop, int layout, const double *a_cur,
                                                   const double *invd, double *rho_out,
                                                   double *u_out, double *partial,
                                                   PairTable<typename St<S>::R> t,
                                                   StepScalars<typename St<S>::R> s) {
    using R = typename St<S>::R;
    using T = typename St<S>::T;
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    double ux_d = 0.0, rho_d = 0.0;
    if (n < (uint32_t)s.nodes) {
        int i, j, k;
        node_ijk(n, s.nx, s.ny, i, j, k);
        const GlobalPop<T> A{(T *)pop};
        const Ix own{aos_base<SET::V>(n), 0u, 0u};
        T raw[SET::V];
        if (layout == kStreamed) {
            read_local<SET>(A, own, raw);
        } else {
            const Nbr3<SET, false> nb(s, i, j, k);
            if (layout == kLocal)
                read_pull3<SET, true>(A, nb, own, raw);
            else
                read_pull3<SET, false>(A, nb, own, raw);
        }
        R d[SET::V];
        complete3d<SET, S>(raw, a_cur, invd, t, s, i, j, k, d);
        const auto m = moments3d<SET, R>(d, s, t.c);
        rho_d = s.rho0d + (double)m.drho;
        ux_d = (double)m.ux;
        if (rho_out) rho_out[n] = rho_d;
        if (u_out) {
            u_out[3 * n] = (double)m.ux;
            u_out[3 * n + 1] = (double)m.uy;
            u_out[3 * n + 2] = (double)m.uz;
        }
    }
    block_sum2(ux_d, rho_d, partial);
}

// init / import: write the node's own slots (kLocal or kDirect)
template <class SET, Storage S>
__device__ __forceinline__ void store_own3d(typename St<S>::T *A, int layout, double *a_out,
                                              const PairTable<typename St<S>::R> &t,
                                              const StepScalars<typename St<S>::R> &s, int i,
                                              int j, int k, const typename St<S>::R (&d)[SET::V],
                                              uint32_t step) {
    using T = typename St<S>::T;
    const uint32_t n = ((uint32_t)k * s.ny + j) * s.nx + i;
    T v[SET::V];
    encode_all<SET, S, false>(d, t, n, step, v);
    if (layout == kLocal)
        write_own<SET, true, false>(A, aos_base<SET::V>(n), v);
    else
        write_own<SET, false, false>(A, aos_base<SET::V>(n), v);
    wall_partials3d<SET, S>(v, t, s, i, j, k, a_out);
}

template <class SET, Storage S>
__global__ __launch_bounds__(256) void k_init3d(void *dst, int layout, double *a_out,
                                                const double *rho_in, const double *u_in,
                                                PairTable<typename St<S>::R> t,
                                                StepScalars<typename St<S>::R> s, uint32_t step) {
    using R = typename St<S>::R;
    using T = typename St<S>::T;
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (uint32_t)s.nodes) return;
    int i, j, k;
    node_ijk(n, s.nx, s.ny, i, j, k);
    const double rho = rho_in ? rho_in[n] : s.rho0d;
    R ux = 0, uy = 0, uz = 0;
    if (u_in) {
        ux = (R)u_in[3 * n];
        uy = (R)u_in[3 * n + 1];
        uz = (R)u_in[3 * n + 2];
    }
    R d[SET::V];
    equilibrium_dev<SET, R>(t, s, rho, ux, uy, uz, d);
    store_own3d<SET, S>((T *)dst, layout, a_out, t, s, i, j, k, d, step);
}

template <class SET, Storage S>
__global__ __launch_bounds__(256) void k_import3d(void *dst, int layout, double *a_out,
                                                  const double *in,
                                                  PairTable<typename St<S>::R> t,
                                                  StepScalars<typename St<S>::R> s, uint32_t step) {
    using R = typename St<S>::R;
    using T = typename St<S>::T;
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (uint32_t)s.nodes) return;
    int i, j, k;
    node_ijk(n, s.nx, s.ny, i, j, k);
    R d[SET::V];
    import_node<SET, R>(in, t, (uint32_t)s.nodes, n, d);
    store_own3d<SET, S>((T *)dst, layout, a_out, t, s, i, j, k, d, step);
}

// canonical FP64 export [alpha][node] of the post-collision populations
template <class SET, Storage S>
__global__ __launch_bounds__(256) void k_export3d(const void *pop, int layout, double *out,
                                                  PairTable<typename St<S>::R> t,
                                                  StepScalars<typename St<S>::R> s) {
    using T = typename St<S>::T;
    constexpr int NR = SET::NR;
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (uint32_t)s.nodes) return;
    int i, j, k;
    node_ijk(n, s.nx, s.ny, i, j, k);
    const uint32_t nodes = (uint32_t)s.nodes;
    const GlobalPop<T> A{(T *)pop};
    const Ix own{aos_base<SET::V>(n), 0u, 0u};
    const Nbr3<SET, false> nb(s, i, j, k);
    if constexpr (NR) out[n] = stored_value<S>(A.ld(own), t.wrd0);
    for_pairs<SET::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        Ix hp, hm;
        if (layout == kLocal) {
            hp = slot_of(own, NR + 2 * p + 1);
            hm = slot_of(own, NR + 2 * p);
        } else if (layout == kDirect) {
            hp = slot_of(own, NR + 2 * p);
            hm = slot_of(own, NR + 2 * p + 1);
        } else {
            hp = home3d<SET, p, true, false, GlobalPop<T>>(nb, own, j, k, s.ny, s.nz);
            hm = home3d<SET, p, false, false, GlobalPop<T>>(nb, own, j, k, s.ny, s.nz);
        }
        out[(uint32_t)(NR + 2 * p) * nodes + n] = stored_value<S>(A.ld(hp), t.wrd[p]);
        out[(uint32_t)(NR + 2 * p + 1) * nodes + n] = stored_value<S>(A.ld(hm), t.wrd[p]);
    });
}

template <class SET, Storage S>
struct L3 {
    using R = typename St<S>::R;
    template <int KIND>
    static void launch_step(const StepBuffers &b, const PairTable<R> &t, const StepScalars<R> &s,
                            hipStream_t st, uint32_t stp) {
        const dim3 g(blocks_for(s.nodes)), bl(256);
        // aligned rows: blocks of up to 256 nodes of one row (nx % 64 == 0)
        const unsigned tb = s.nx % 256 == 0 ? 256u : (s.nx % 128 == 0 ? 128u : 64u);
        const dim3 g2((unsigned)s.nx / tb, (unsigned)(s.ny * s.nz)), bl2(tb);
        if (s.aligned_rows && s.stream_stores)
            hipLaunchKernelGGL((k_step3d<SET, S, true, true, KIND>), g2, bl2, 0, st, b, t, s, stp);
        else if (s.aligned_rows)
            hipLaunchKernelGGL((k_step3d<SET, S, true, false, KIND>), g2, bl2, 0, st, b, t, s, stp);
        else
            hipLaunchKernelGGL((k_step3d<SET, S, false, false, KIND>), g, bl, 0, st, b, t, s, stp);
    }
    static int step(const StepBuffers &b, const void *tab, const void *sc, hipStream_t st,
                    uint32_t stp) {
        const auto &t = *(const PairTable<R> *)tab;
        const auto &s = *(const StepScalars<R> *)sc;
        if (b.layout == kLocal)
            launch_step<kGatherScatter3>(b, t, s, st, stp);
        else if (b.layout == kStreamed)
            launch_step<kNodeLocal3>(b, t, s, st, stp);
        else
            launch_step<kPingPong3>(b, t, s, st, stp);
        return hip_ok(hipGetLastError(), "3D step kernel launch");
    }
    static int init(void *dst, int layout, double *a_out, const double *rho, const double *u,
                    const void *tab, const void *sc, hipStream_t st, uint32_t stp) {
        const auto &t = *(const PairTable<R> *)tab;
        const auto &s = *(const StepScalars<R> *)sc;
        hipLaunchKernelGGL((k_init3d<SET, S>), dim3(blocks_for(s.nodes)), dim3(256), 0, st, dst,
                           layout, a_out, rho, u, t, s, stp);
        return hip_ok(hipGetLastError(), "3D init kernel launch");
    }
    static int observe(const void *pop, int layout, const double *a_cur, const double *invd,
                       double *rho, double *u, double *partial, const void *tab, const void *sc,
                       hipStream_t st) {
        const auto &t = *(const PairTable<R> *)tab;
        const auto &s = *(const StepScalars<R> *)sc;
        hipLaunchKernelGGL((k_observe3d<SET, S>), dim3(blocks_for(s.nodes)), dim3(256), 0, st,
                           pop, layout, a_cur, invd, rho, u, partial, t, s);
        return hip_ok(hipGetLastError(), "3D observe kernel launch");
    }
    static int exportp(const void *pop, int layout, double *out, const void *tab, const void *sc,
                       hipStream_t st) {
        const auto &t = *(const PairTable<R> *)tab;
        const auto &s = *(const StepScalars<R> *)sc;
        hipLaunchKernelGGL((k_export3d<SET, S>), dim3(blocks_for(s.nodes)), dim3(256), 0, st, pop,
                           layout, out, t, s);
        return hip_ok(hipGetLastError(), "3D export kernel launch");
    }
    static int importp(void *dst, int layout, double *a_out, const double *in, const void *tab,
                       const void *sc, hipStream_t st, uint32_t stp) {
        const auto &t = *(const PairTable<R> *)tab;
        const auto &s = *(const StepScalars<R> *)sc;
        hipLaunchKernelGGL((k_import3d<SET, S>), dim3(blocks_for(s.nodes)), dim3(256), 0, st,
                           dst, layout, a_out, in, t, s, stp);
        return hip_ok(hipGetLastError(), "3D import kernel launch");
    }
    static constexpr Launch table{&step, &init, &observe, &exportp, &importp, nullptr, nullptr};
};

#define LBM_3D(SET)                                                           \
    {SET::ID, Storage::F64, &L3<SET, Storage::F64>::table},                   \
        {SET::ID, Storage::F32, &L3<SET, Storage::F32>::table},               \
        {SET::ID, Storage::F32RAW, &L3<SET, Storage::F32RAW>::table},         \
        {SET::ID, Storage::F16DEV, &L3<SET, Storage::F16DEV>::table}

const Launch *find_launch_3d(int set_id, Storage st) {
    static const Entry entries[] = {LBM_3D(SetD3V39), LBM_3D(SetD3V15), LBM_3D(SetD3V96)};
    for (const auto &e : entries)
        if (e.id == set_id && e.s == st) return e.l;
    return nullptr;
}

}  // namespace lbm
