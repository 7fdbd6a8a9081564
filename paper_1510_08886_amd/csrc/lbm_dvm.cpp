// Discrete velocity models (Section II of the paper): velocity groups, the
// moment conditions of a lattice Gauss-Hermite quadrature, and the lattice
// speed c* at which a minimal set of groups becomes a quadrature.
//
// Formulation used here: with all weights of a group equal (Eq. wdach) and the
// groups invariant under signed permutations, the quadrature conditions
// (Eqs. genQua / orth) reduce to one equation per even, sorted monomial
// exponent a (a_1 >= a_2 >= ... , all even, |a| <= Q):
//     sum_g wbar_g c^{|a|} M_g(a) = prod_d (a_d - 1)!!,   M_g(a) = sum_{e in S_g} e^a,
// which are linear in wbar for fixed c. A minimal DVM (Eq. dimker) is a c at
// which this overdetermined system becomes consistent. Square systems
// (equations = groups + 1) are solved as roots of det[A(c) | b]; others by
// minimising the least-squares residual over c. All of it in long double.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <set>

#include "lbm_internal.h"

using ld = long double;

namespace lbm {

namespace {

using Vec = std::vector<int32_t>;

std::vector<Vec> signed_permutations(const Vec &gen) {
    const int d = (int)gen.size();
    std::vector<int> perm(d);
    for (int k = 0; k < d; ++k) perm[k] = k;
    std::set<Vec> out;
    do {
        for (int mask = 0; mask < (1 << d); ++mask) {
            Vec v(d);
            for (int k = 0; k < d; ++k) v[k] = ((mask >> k) & 1 ? -1 : 1) * gen[perm[k]];
            out.insert(v);
        }
    } while (std::next_permutation(perm.begin(), perm.end()));
    return std::vector<Vec>(out.begin(), out.end());
}

ld double_factorial_odd(int a) {  // (a-1)!! for even a >= 0
    ld r = 1;
    for (int k = a - 1; k > 1; k -= 2) r *= k;
    return r;
}

ld gauss_moment(const std::vector<int> &a) {
    ld r = 1;
    for (int x : a) {
        if (x & 1) return 0;
        r *= double_factorial_odd(x);
    }
    return r;
}

// even exponents, non-increasing, total <= Q
void even_sorted(int dim, int Q, std::vector<std::vector<int>> &out) {
    std::function<void(std::vector<int> &, int, int)> rec = [&](std::vector<int> &cur, int maxv,
                                                               int left) {
        if ((int)cur.size() == dim) {
            out.push_back(cur);
            return;
        }
        for (int v = std::min(maxv, left) & ~1; v >= 0; v -= 2) {
            cur.push_back(v);
            rec(cur, v, left - v);
            cur.pop_back();
        }
    };
    std::vector<int> cur;
    rec(cur, Q & ~1, Q);
}

struct MomentSystem {
    int G = 0, E = 0;
    std::vector<int> deg;          // |a| per equation
    std::vector<ld> gm;            // Gaussian moment per equation
    std::vector<std::vector<ld>> M;  // E x G orbit moment sums
    std::vector<int> sizes;
};

MomentSystem build_system(int dim, const std::vector<Vec> &gens, int Q) {
    MomentSystem s;
    s.G = (int)gens.size();
    std::vector<std::vector<int>> exps;
    even_sorted(dim, Q, exps);
    s.E = (int)exps.size();
    std::vector<std::vector<Vec>> orbits;
    for (const auto &g : gens) orbits.push_back(signed_permutations(g));
    for (const auto &o : orbits) s.sizes.push_back((int)o.size());
    for (const auto &a : exps) {
        int dsum = 0;
        for (int x : a) dsum += x;
        s.deg.push_back(dsum);
        s.gm.push_back(gauss_moment(a));
        std::vector<ld> row(s.G);
        for (int g = 0; g < s.G; ++g) {
            ld sum = 0;
            for (const auto &e : orbits[g]) {
                ld p = 1;
                for (int k = 0; k < dim; ++k)
                    for (int q = 0; q < a[k]; ++q) p *= e[k];
                sum += p;
            }
            row[g] = sum;
        }
        s.M.push_back(row);
    }
    return s;
}

// Row-normalised augmented matrix [A(c) | b]
void augmented(const MomentSystem &s, ld c, std::vector<std::vector<ld>> &Ab) {
    Ab.assign(s.E, std::vector<ld>(s.G + 1));
    for (int r = 0; r < s.E; ++r) {
        const ld cp = std::pow(c, (ld)s.deg[r]);
        for (int g = 0; g < s.G; ++g) Ab[r][g] = s.M[r][g] * cp / s.gm[r];
        Ab[r][s.G] = 1;
    }
}

ld det_square(std::vector<std::vector<ld>> m) {
    const int n = (int)m.size();
    ld det = 1;
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int r = k + 1; r < n; ++r)
            if (std::fabs(m[r][k]) > std::fabs(m[piv][k])) piv = r;
        if (m[piv][k] == 0) return 0;
        if (piv != k) {
            std::swap(m[piv], m[k]);
            det = -det;
        }
        det *= m[k][k];
        for (int r = k + 1; r < n; ++r) {
            const ld f = m[r][k] / m[k][k];
            for (int q = k; q < n; ++q) m[r][q] -= f * m[k][q];
        }
    }
    return det;
}

// Least squares A w = b by Householder QR; returns the residual norm.
ld least_squares(const MomentSystem &s, ld c, std::vector<ld> &w) {
    std::vector<std::vector<ld>> Ab;
    augmented(s, c, Ab);
    const int m = s.E, n = s.G;
    for (int k = 0; k < n && k < m; ++k) {
        ld norm = 0;
        for (int r = k; r < m; ++r) norm += Ab[r][k] * Ab[r][k];
        norm = std::sqrt(norm);
        if (norm == 0) continue;
        const ld alpha = Ab[k][k] > 0 ? -norm : norm;
        std::vector<ld> v(m, 0);
        v[k] = Ab[k][k] - alpha;
        for (int r = k + 1; r < m; ++r) v[r] = Ab[r][k];
        ld vn = 0;
        for (int r = k; r < m; ++r) vn += v[r] * v[r];
        if (vn == 0) continue;
        for (int q = k; q <= n; ++q) {
            ld dot = 0;
            for (int r = k; r < m; ++r) dot += v[r] * Ab[r][q];
            const ld f = 2 * dot / vn;
            for (int r = k; r < m; ++r) Ab[r][q] -= f * v[r];
        }
    }
    w.assign(n, 0);
    for (int k = n - 1; k >= 0; --k) {
        ld acc = Ab[k][n];
        for (int q = k + 1; q < n; ++q) acc -= Ab[k][q] * w[q];
        w[k] = Ab[k][k] != 0 ? acc / Ab[k][k] : 0;
    }
    ld res = 0;
    for (int r = n; r < m; ++r) res += Ab[r][n] * Ab[r][n];
    return std::sqrt(res);
}

}  // namespace

// returns all c in [lo, hi] with a consistent system, with their weights
static void find_roots(const MomentSystem &s, ld lo, ld hi,
                       std::vector<std::pair<ld, std::vector<ld>>> &roots) {
    const int n = 20000;
    if (s.E < s.G + 1) return;  // not minimal: a family of solutions, no isolated c*
    if (s.E == s.G + 1) {
        auto f = [&](ld c) {
            std::vector<std::vector<ld>> Ab;
            augmented(s, c, Ab);
            return det_square(Ab);
        };
        ld cprev = lo, fprev = f(lo);
        for (int k = 1; k <= n; ++k) {
            const ld c = lo + (hi - lo) * k / n;
            const ld fc = f(c);
            if ((fprev < 0) != (fc < 0) || fc == 0) {
                ld a = cprev, b = c, fa = fprev;
                for (int it = 0; it < 200 && b - a > 1e-19L * b; ++it) {
                    const ld m = 0.5L * (a + b);
                    const ld fm = f(m);
                    if ((fa < 0) != (fm < 0)) {
                        b = m;
                    } else {
                        a = m;
                        fa = fm;
                    }
                }
                const ld root = 0.5L * (a + b);
                std::vector<ld> w;
                const ld res = least_squares(s, root, w);
                if (res < 1e-12L) roots.push_back({root, w});
            }
            cprev = c;
            fprev = fc;
        }
        return;
    }
    // overdetermined: V-shaped residual minima
    std::vector<ld> cs(n + 1), rs(n + 1);
    std::vector<ld> w;
    for (int k = 0; k <= n; ++k) {
        cs[k] = lo + (hi - lo) * k / n;
        rs[k] = least_squares(s, cs[k], w);
    }
    for (int k = 1; k < n; ++k) {
        if (!(rs[k] <= rs[k - 1] && rs[k] <= rs[k + 1])) continue;
        ld a = cs[k - 1], b = cs[k + 1];
        const ld gr = 0.6180339887498948482L;
        ld x1 = b - gr * (b - a), x2 = a + gr * (b - a);
        ld f1 = least_squares(s, x1, w), f2 = least_squares(s, x2, w);
        for (int it = 0; it < 200 && b - a > 1e-19L * b; ++it) {
            if (f1 < f2) {
                b = x2;
                x2 = x1;
                f2 = f1;
                x1 = b - gr * (b - a);
                f1 = least_squares(s, x1, w);
            } else {
                a = x1;
                x1 = x2;
                f1 = f2;
                x2 = a + gr * (b - a);
                f2 = least_squares(s, x2, w);
            }
        }
        const ld root = 0.5L * (a + b);
        const ld res = least_squares(s, root, w);
        if (res < 1e-12L) roots.push_back({root, w});
    }
}

}  // namespace lbm

using namespace lbm;

extern "C" int lbm_dvm_solve(int dim, int n_groups, const int32_t *gen, int Q, double c_lo,
                             double c_hi, double *c_out, double *w_group_out, int *n_vel_out) {
    if (dim < 2 || dim > 3 || n_groups < 1 || !gen || Q < 1 || !(c_lo > 0) || !(c_hi > c_lo))
        return fail(LBM_E_INVALID, "lbm_dvm_solve: bad arguments");
    std::vector<Vec> gens;
    for (int g = 0; g < n_groups; ++g) gens.push_back(Vec(gen + g * dim, gen + (g + 1) * dim));
    MomentSystem s = build_system(dim, gens, Q);
    std::vector<std::pair<ld, std::vector<ld>>> roots;
    find_roots(s, c_lo, c_hi, roots);
    std::sort(roots.begin(), roots.end(),
              [](const auto &a, const auto &b) { return a.first < b.first; });
    for (auto &r : roots) {
        bool pos = true;
        for (ld x : r.second) pos = pos && x > 0;
        if (!pos) continue;
        if (c_out) *c_out = (double)r.first;
        if (w_group_out)
            for (int g = 0; g < n_groups; ++g) w_group_out[g] = (double)r.second[g];
        if (n_vel_out) {
            int V = 0;
            for (int x : s.sizes) V += x;
            *n_vel_out = V;
        }
        return LBM_OK;
    }
    return fail(LBM_E_QUADRATURE, "lbm_dvm_solve: no positive-weight quadrature in range");
}

extern "C" int lbm_dvm_create(int dim, int n_groups, const int32_t *gen, const double *w_group,
                              double c, int Q, lbm_dvm_t **out) {
    if (!out || dim < 2 || dim > 3 || n_groups < 1 || !gen || !w_group || !(c > 0) || Q < 1)
        return fail(LBM_E_INVALID, "lbm_dvm_create: bad arguments");
    *out = nullptr;
    // union of the groups; each velocity once
    std::map<Vec, double> wmap;
    for (int g = 0; g < n_groups; ++g) {
        if (!(w_group[g] > 0)) return fail(LBM_E_INVALID, "lbm_dvm_create: weights must be positive");
        for (const auto &e : signed_permutations(Vec(gen + g * dim, gen + (g + 1) * dim))) {
            if (wmap.count(e)) return fail(LBM_E_INVALID, "lbm_dvm_create: groups overlap");
            wmap[e] = w_group[g];
        }
    }
    auto *d = new Dvm();
    d->dim = dim;
    d->Q = Q;
    d->c = c;
    d->n_groups = n_groups;
    auto push = [&](const Vec &e, double w) {
        for (int k = 0; k < 3; ++k) d->vel.push_back(k < dim ? e[k] : 0);
        d->w.push_back(w);
        for (int k = 0; k < dim; ++k) d->halo = std::max(d->halo, std::abs(e[k]));
    };
    const Vec zero(dim, 0);
    if (wmap.count(zero)) {
        push(zero, wmap[zero]);
        d->n_rest = 1;
    }
    for (const auto &kv : wmap) {
        const Vec &e = kv.first;
        int first = 0;
        for (int k = 0; k < dim && first == 0; ++k) first = e[k];
        if (first <= 0) continue;  // emit each pair from its "positive" member
        Vec m(dim);
        for (int k = 0; k < dim; ++k) m[k] = -e[k];
        push(e, kv.second);
        push(m, wmap.at(m));
    }
    d->V = (int)d->w.size();
    // moment check to degree Q
    std::function<void(std::vector<int> &, int)> rec;
    ld worst = 0;
    rec = [&](std::vector<int> &a, int left) {
        if ((int)a.size() == dim) {
            ld q = 0;
            for (int v = 0; v < d->V; ++v) {
                ld p = d->w[v];
                for (int k = 0; k < dim; ++k)
                    for (int t = 0; t < a[k]; ++t) p *= (ld)c * d->vel[3 * v + k];
                q += p;
            }
            const ld want = gauss_moment(a);
            worst = std::max(worst, std::fabs(q - want) / std::max((ld)1, std::fabs(want)));
            return;
        }
        for (int x = 0; x <= left; ++x) {
            a.push_back(x);
            rec(a, left - x);
            a.pop_back();
        }
    };
    std::vector<int> a;
    rec(a, Q);
    if (!(worst < 1e-12L)) {
        delete d;
        return fail(LBM_E_QUADRATURE, "lbm_dvm_create: velocity set is not a quadrature of order Q");
    }
    *out = reinterpret_cast<lbm_dvm_t *>(d);
    return LBM_OK;
}

extern "C" int lbm_dvm_destroy(lbm_dvm_t *dvm) {
    delete reinterpret_cast<Dvm *>(dvm);
    return LBM_OK;
}

extern "C" int lbm_dvm_info(const lbm_dvm_t *dvm, int *V, int32_t *vel, double *w, double *c) {
    if (!dvm) return fail(LBM_E_INVALID, "lbm_dvm_info: null handle");
    const Dvm *d = reinterpret_cast<const Dvm *>(dvm);
    if (V) *V = d->V;
    if (vel)
        for (int v = 0; v < d->V; ++v)
            for (int k = 0; k < d->dim; ++k) vel[v * d->dim + k] = d->vel[3 * v + k];
    if (w)
        for (int v = 0; v < d->V; ++v) w[v] = d->w[v];
    if (c) *c = d->c;
    return LBM_OK;
}
