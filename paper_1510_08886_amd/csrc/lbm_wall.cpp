// Wall-moment diagnostics of a velocity set (Section IV of the paper): how well
// the quadrature over the velocities leaving a wall reproduces the half-space
// moments of the Maxwellian that the diffuse Maxwell wall emits. Host only.
#include <cmath>
#include <cstring>
#include <vector>

#include "lbm_internal.h"

namespace lbm {
namespace {

using ld = long double;

// (m - 1)!! with (-1)!! = 1
ld odd_factorial(int m) {
    ld r = 1;
    for (int k = m - 1; k > 1; k -= 2) r *= k;
    return r;
}

// integral over the whole line of the unit Gaussian density times x^m
ld full_line(int m) { return (m % 2) ? 0.0L : odd_factorial(m); }

// integral over x > 0 of the unit Gaussian density times x^m: half the full
// moment for even m; (m - 1)!! / sqrt(2 pi) for odd m
ld half_line(int m) {
    if (m % 2 == 0) return odd_factorial(m) / 2;
    return odd_factorial(m) / std::sqrt(2.0L * 3.14159265358979323846264338327950288L);
}

struct Triple {
    int mx, my, mz;
};

// Non-trivial wall moments (Eq. nontriv), ordered as in Eqs. defT / defb:
// rank n ascending, then m_z descending, then m_x descending.
std::vector<Triple> components(int Q, int dim) {
    std::vector<Triple> out;
    for (int n = 0; n <= Q; ++n)
        for (int mz = n; mz >= 0; --mz) {
            if (mz != 0 && mz % 2 == 0) continue;
            for (int mx = n - mz; mx >= 0; --mx) {
                const int my = n - mz - mx;
                if (mx % 2 || my % 2 || my > mx || (dim == 2 && my != 0)) continue;
                out.push_back({mx, my, mz});
            }
        }
    return out;
}

struct WallQuad {
    const Dvm &d;
    int ax, ay, az;  // velocity components used as tangential x, y and normal z
    ld exact(const Triple &t) const {
        return full_line(t.mx) * (d.dim == 3 ? full_line(t.my) : 1.0L) * half_line(t.mz);
    }
    // sum over velocities pointing into the fluid (e_z > 0); `absval` sums |terms|
    ld quad(const Triple &t, bool absval = false) const {
        ld s = 0;
        for (int v = 0; v < d.V; ++v) {
            const int *e = &d.vel[3 * v];
            if (e[az] <= 0) continue;
            ld p = d.w[v];
            const ld c = d.c;
            for (int k = 0; k < t.mx; ++k) p *= c * e[ax];
            if (ay >= 0)
                for (int k = 0; k < t.my; ++k) p *= c * e[ay];
            for (int k = 0; k < t.mz; ++k) p *= c * e[az];
            s += absval ? std::fabs(p) : p;
        }
        return s;
    }
    bool exact_to(const Triple &t, ld tol) const {
        const ld a = exact(t), b = quad(t);
        const ld scale = a != 0 ? std::fabs(a) : quad(t, true);
        return std::fabs(b - a) <= tol * std::max(scale, (ld)1e-300L);
    }
};

constexpr ld kExactTol = 1e-10L;

}  // namespace
}  // namespace lbm

using namespace lbm;

extern "C" int lbm_dvm_wall_errors(const lbm_dvm_t *dvm, int normal_axis, int cap, int32_t *exps,
                                   double *w_exact, double *w_dvm, double *sigma,
                                   lbm_wall_report_t *report) {
    if (!dvm) return fail(LBM_E_INVALID, "lbm_dvm_wall_errors: null handle");
    const Dvm &d = *reinterpret_cast<const Dvm *>(dvm);
    if (normal_axis < 0 || normal_axis >= d.dim)
        return fail(LBM_E_INVALID, "lbm_dvm_wall_errors: normal axis out of range");
    int axes[2], na = 0;
    for (int k = 0; k < d.dim; ++k)
        if (k != normal_axis) axes[na++] = k;
    WallQuad wq{d, axes[0], d.dim == 3 ? axes[1] : -1, normal_axis};
    const auto comps = components(d.Q, d.dim);
    const int L = (int)comps.size();
    if (L > 64) return fail(LBM_E_UNSUPPORTED, "lbm_dvm_wall_errors: more than 64 wall moments");
    const bool want_arrays = exps || w_exact || w_dvm || sigma;
    if (want_arrays && cap < L)
        return fail(LBM_E_NO_MEMORY, "lbm_dvm_wall_errors: arrays shorter than the moment count");
    ld num = 0, den = 0;
    uint64_t index = 0;
    for (int k = 0; k < L; ++k) {
        const Triple &t = comps[k];
        const ld a = wq.exact(t), b = wq.quad(t);
        const ld s = (b - a) / a;  // sign of the printed tables: (W^DVM - W) / W
        const ld wt = std::exp(-(ld)(t.mx + t.my + t.mz));
        num += std::fabs(s) * wt;
        den += wt;
        if (std::fabs(s) <= kExactTol) index |= (uint64_t)1 << k;
        if (exps) {
            exps[3 * k] = t.mx;
            exps[3 * k + 1] = t.my;
            exps[3 * k + 2] = t.mz;
        }
        if (w_exact) w_exact[k] = (double)a;
        if (w_dvm) w_dvm[k] = (double)b;
        if (sigma) sigma[k] = (double)s;
    }
    // wall accuracy order: every moment of rank <= Lambda exact, trivial ones included
    int order = -1;
    for (int n = 0; n <= d.Q; ++n) {
        bool ok = true;
        for (int mx = 0; mx <= n && ok; ++mx)
            for (int my = 0; my <= (d.dim == 3 ? n - mx : 0) && ok; ++my)
                ok = wq.exact_to({mx, my, n - mx - my}, kExactTol);
        if (!ok) break;
        order = n;
    }
    if (report) {
        report->n_components = L;
        report->lambda_order = order;
        report->lambda_index = index;
        report->sigma_sigma = (double)(num / den);
    }
    return LBM_OK;
}
