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
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <set>
#include <mutex>
#include <thread>

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

// ---------------------------------------------------------------------------
// Enumeration of the minimal DVMs inside an energy sphere (Section II.B:
// the stencil energy E = (1 / 2c^2) sum |xi|^2 = (1/2) sum |e|^2 <= E_max).
//
// A candidate is a set of distinct velocity groups (orbits of integer
// generators under signed permutations) of total energy <= E_max. With x =
// 1 / c^2 the moment conditions read M w = b(x), b_a(x) = gm(a) x^{|a|/2},
// with the integer orbit-sum matrix M (equations x groups) independent of c.
// A minimal DVM (Eq. dimker) has a unique weight vector (M of full column
// rank G) at an isolated c*: b(x) must lie in the column space of M, i.e.
// y.b(x) = 0 for every y of the left null space of M (dimension
// equations - G >= 1), a polynomial in x of degree <= Q / 2 per y; c* are
// the positive common roots. Only positive weights are kept.
// ---------------------------------------------------------------------------
namespace {

using Poly = std::vector<ld>;   // coefficients of x^0, x^1, ...

ld poly_eval(const Poly &p, ld x) {
    ld r = 0;
    for (size_t k = p.size(); k-- > 0;) r = r * x + p[k];
    return r;
}

Poly poly_deriv(const Poly &p) {
    Poly d;
    for (size_t k = 1; k < p.size(); ++k) d.push_back(p[k] * (ld)k);
    return d;
}

void poly_trim(Poly &p) {
    ld scale = 0;
    for (ld c : p) scale = std::max(scale, std::fabs(c));
    while (!p.empty() && std::fabs(p.back()) <= 1e-15L * scale) p.pop_back();
}

// real roots of p in (lo, hi), each bracketed between consecutive critical
// points (roots of p') and bisected; tangent roots are not returned
void poly_roots(Poly p, ld lo, ld hi, std::vector<ld> &out) {
    poly_trim(p);
    if (p.size() < 2) return;
    std::vector<ld> crit;
    poly_roots(poly_deriv(p), lo, hi, crit);
    std::vector<ld> pts{lo};
    for (ld c : crit) pts.push_back(c);
    pts.push_back(hi);
    for (size_t k = 0; k + 1 < pts.size(); ++k) {
        ld a = pts[k], b = pts[k + 1];
        ld fa = poly_eval(p, a), fb = poly_eval(p, b);
        if (fa == 0) {
            if (k == 0) continue;
            out.push_back(a);
            continue;
        }
        if ((fa < 0) == (fb < 0)) continue;
        for (int it = 0; it < 200 && b - a > 1e-19L * b; ++it) {
            const ld m = 0.5L * (a + b), fm = poly_eval(p, m);
            if ((fa < 0) == (fm < 0)) {
                a = m;
                fa = fm;
            } else {
                b = m;
            }
        }
        out.push_back(0.5L * (a + b));
    }
    std::sort(out.begin(), out.end());
}

struct Generator {
    Vec g;
    int size = 0, energy2 = 0;   // orbit size, 2 E of the group
};

// canonical generators (0 <= g_1 <= ... <= g_D) of groups with energy <= emax
std::vector<Generator> generators(int dim, int emax) {
    std::vector<Generator> out;
    const int r = (int)std::sqrt(2.0 * emax) + 1;
    std::function<void(Vec &, int)> rec = [&](Vec &cur, int from) {
        if ((int)cur.size() == dim) {
            Generator G;
            G.g = cur;
            G.size = (int)signed_permutations(cur).size();
            int n2 = 0;
            for (int x : cur) n2 += x * x;
            G.energy2 = G.size * n2;
            if (G.energy2 <= 2 * emax) out.push_back(G);
            return;
        }
        for (int v = from; v <= r; ++v) {
            cur.push_back(v);
            rec(cur, v);
            cur.pop_back();
        }
    };
    Vec cur;
    rec(cur, 0);
    std::stable_sort(out.begin(), out.end(),
                     [](const Generator &a, const Generator &b) { return a.energy2 < b.energy2; });
    return out;
}

struct Found {
    int V, E;
    std::vector<int> groups;   // indices into the generator list
    ld c;
    std::vector<ld> w;
};

// Minimal DVMs of one candidate: cols[q] are the orbit-sum columns of its
// groups (moment equations in rows), deg/gm per row.
void minimal_models(const std::vector<const std::vector<ld> *> &cols, const std::vector<int> &deg,
                    const std::vector<ld> &gm, ld x_lo, ld x_hi,
                    std::vector<std::pair<ld, std::vector<ld>>> &models) {
    const int n = (int)deg.size(), G = (int)cols.size();
    if (G >= n) return;                  // no isolated c*: a family of solutions or none
    // rows scaled to unit max norm
    std::vector<ld> sc(n, 1);
    std::vector<std::vector<ld>> A(n, std::vector<ld>(G));
    for (int r = 0; r < n; ++r) {
        ld m = 0;
        for (int q = 0; q < G; ++q) m = std::max(m, std::fabs((*cols[q])[r]));
        sc[r] = m > 0 ? 1 / m : 1;
        for (int q = 0; q < G; ++q) A[r][q] = (*cols[q])[r] * sc[r];
    }
    // Householder QR, Q accumulated explicitly (n <= 16)
    std::vector<std::vector<ld>> Qm(n, std::vector<ld>(n, 0));
    for (int r = 0; r < n; ++r) Qm[r][r] = 1;
    ld rmax = 0;
    for (int k = 0; k < G; ++k) {
        ld norm = 0;
        for (int r = k; r < n; ++r) norm += A[r][k] * A[r][k];
        norm = std::sqrt(norm);
        rmax = std::max(rmax, norm);
        if (norm <= 1e-14L * std::max(rmax, (ld)1)) return;   // rank deficient
        const ld alpha = A[k][k] > 0 ? -norm : norm;
        std::vector<ld> v(n, 0);
        v[k] = A[k][k] - alpha;
        for (int r = k + 1; r < n; ++r) v[r] = A[r][k];
        ld vn = 0;
        for (int r = k; r < n; ++r) vn += v[r] * v[r];
        for (int q = k; q < G; ++q) {
            ld dot = 0;
            for (int r = k; r < n; ++r) dot += v[r] * A[r][q];
            const ld f = 2 * dot / vn;
            for (int r = k; r < n; ++r) A[r][q] -= f * v[r];
        }
        for (int q = 0; q < n; ++q) {   // Qm <- Qm H_k (columns are Q's)
            ld dot = 0;
            for (int r = k; r < n; ++r) dot += Qm[q][r] * v[r];
            const ld f = 2 * dot / vn;
            for (int r = k; r < n; ++r) Qm[q][r] -= f * v[r];
        }
    }
    for (int k = 0; k < G; ++k)
        if (std::fabs(A[k][k]) <= 1e-12L * rmax) return;      // rank deficient
    // left null space: columns G..n-1 of Q; polynomials y.b(x) in x
    const int dmax = *std::max_element(deg.begin(), deg.end()) / 2;
    std::vector<Poly> polys;
    for (int k = G; k < n; ++k) {
        Poly p(dmax + 1, 0);
        for (int r = 0; r < n; ++r) p[deg[r] / 2] += Qm[r][k] * sc[r] * gm[r];
        polys.push_back(p);
    }
    std::vector<ld> roots;
    poly_roots(polys[0], x_lo, x_hi, roots);
    for (ld x : roots) {
        bool common = true;
        for (size_t k = 1; k < polys.size() && common; ++k) {
            ld mag = 0;
            for (int j = 0; j <= dmax; ++j) mag += std::fabs(polys[k][j]) * std::pow(x, (ld)j);
            common = std::fabs(poly_eval(polys[k], x)) <= 1e-11L * mag;
        }
        if (!common) continue;
        // weights: R w = Q^T (S b)
        std::vector<ld> sb(n);
        for (int r = 0; r < n; ++r) sb[r] = sc[r] * gm[r] * std::pow(x, (ld)(deg[r] / 2));
        std::vector<ld> qb(G, 0);
        for (int k = 0; k < G; ++k)
            for (int r = 0; r < n; ++r) qb[k] += Qm[r][k] * sb[r];
        std::vector<ld> w(G, 0);
        for (int k = G - 1; k >= 0; --k) {
            ld acc = qb[k];
            for (int q = k + 1; q < G; ++q) acc -= A[k][q] * w[q];
            w[k] = acc / A[k][k];
        }
        // positive weights, each well above the rounding of the largest (a
        // weight that vanishes at c* means a smaller stencil is the quadrature)
        ld wmax = 0;
        for (ld v : w) wmax = std::max(wmax, std::fabs(v));
        bool pos = true;
        for (ld v : w) pos = pos && v > 1e-12L * wmax;
        if (!pos) continue;
        // residual of the full system, relative to b
        ld res = 0, bn = 0;
        for (int r = 0; r < n; ++r) {
            ld acc = -sb[r];
            for (int q = 0; q < G; ++q) acc += (*cols[q])[r] * sc[r] * w[q];
            res += acc * acc;
            bn += sb[r] * sb[r];
        }
        if (res > 1e-20L * bn) continue;
        models.push_back({1 / std::sqrt(x), w});
    }
}

}  // namespace

extern "C" int lbm_dvm_enumerate(int dim, int Q, int e_max, int max_groups, int flags,
                                 lbm_dvm_model_t *out, int cap, int *n_out) {
    if (dim < 2 || dim > 3 || Q < 1 || Q > 13 || e_max < 0 || max_groups < 0 || cap < 0 ||
        (cap > 0 && !out) || (flags & ~LBM_ENUM_SCATTERING))
        return fail(LBM_E_INVALID, "lbm_dvm_enumerate: bad arguments");
    std::vector<std::vector<int>> exps;
    even_sorted(dim, Q, exps);
    const int n = (int)exps.size();
    if (max_groups == 0 || max_groups > n - 1) max_groups = n - 1;
    if (max_groups > LBM_MAX_GROUPS)
        return fail(LBM_E_UNSUPPORTED, "lbm_dvm_enumerate: more than 16 groups per stencil");
    std::vector<int> deg;
    std::vector<ld> gm;
    for (const auto &a : exps) {
        int d = 0;
        for (int x : a) d += x;
        deg.push_back(d);
        gm.push_back(gauss_moment(a));
    }
    std::vector<Generator> gens;
    for (const auto &g : generators(dim, e_max)) {
        bool keep = true;
        if (flags & LBM_ENUM_SCATTERING)
            for (int x : g.g) keep = keep && x != 0;
        if (keep) gens.push_back(g);
    }
    std::vector<std::vector<ld>> col(gens.size(), std::vector<ld>(n));
    for (size_t g = 0; g < gens.size(); ++g) {
        const auto orbit = signed_permutations(gens[g].g);
        for (int r = 0; r < n; ++r) {
            ld sum = 0;
            for (const auto &e : orbit) {
                ld p = 1;
                for (int k = 0; k < dim; ++k)
                    for (int q = 0; q < exps[r][k]; ++q) p *= e[k];
                sum += p;
            }
            col[g][r] = sum;
        }
    }
    // c* in [0.02, 50]
    const ld x_lo = 1 / (50.0L * 50.0L), x_hi = 1 / (0.02L * 0.02L);
    // Candidates by depth-first search over generator subsets in energy
    // order; the subtrees of the first generator are shared out to threads.
    std::vector<std::pair<int, int>> tasks;
    for (size_t g1 = 0; g1 < gens.size(); ++g1) {
        tasks.push_back({(int)g1, -1});
        if (max_groups < 2) continue;
        for (size_t g2 = g1 + 1; g2 < gens.size(); ++g2)
            if (gens[g1].energy2 + gens[g2].energy2 <= 2 * e_max) tasks.push_back({(int)g1, (int)g2});
    }
    std::atomic<size_t> next{0};
    std::mutex mu;
    std::vector<Found> found;
    auto worker = [&]() {
        std::vector<Found> mine;
        std::vector<int> pick;
        std::vector<const std::vector<ld> *> cols;
        std::vector<std::pair<ld, std::vector<ld>>> models;
        std::function<void(size_t, int)> rec = [&](size_t from, int e2) {
            models.clear();
            minimal_models(cols, deg, gm, x_lo, x_hi, models);
            for (auto &m : models) {
                Found f;
                f.V = 0;
                for (int g : pick) f.V += gens[g].size;
                f.E = e2 / 2;
                f.groups = pick;
                f.c = m.first;
                f.w = m.second;
                mine.push_back(f);
            }
            if ((int)pick.size() == max_groups) return;
            for (size_t g = from; g < gens.size(); ++g) {
                if (e2 + gens[g].energy2 > 2 * e_max) break;   // sorted by energy
                pick.push_back((int)g);
                cols.push_back(&col[g]);
                rec(g + 1, e2 + gens[g].energy2);
                pick.pop_back();
                cols.pop_back();
            }
        };
        // task t < G: the stencil of generator t alone; then the subtrees
        // below each pair (g1 < g2), in a fixed order
        for (size_t t; (t = next.fetch_add(1)) < tasks.size();) {
            const auto [g1, g2] = tasks[t];
            if (g2 < 0) {
                pick.assign(1, g1);
                cols.assign(1, &col[g1]);
                models.clear();
                minimal_models(cols, deg, gm, x_lo, x_hi, models);
                for (auto &m : models)
                    mine.push_back({gens[g1].size, gens[g1].energy2 / 2, pick, m.first, m.second});
                continue;
            }
            pick.assign({g1, g2});
            cols.assign({&col[g1], &col[g2]});
            rec(g2 + 1, gens[g1].energy2 + gens[g2].energy2);
        }
        std::lock_guard<std::mutex> lk(mu);
        found.insert(found.end(), mine.begin(), mine.end());
    };
    const int nthreads = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (int k = 0; k < nthreads; ++k) pool.emplace_back(worker);
    for (auto &t : pool) t.join();
    std::sort(found.begin(), found.end(), [](const Found &a, const Found &b) {
        if (a.V != b.V) return a.V < b.V;
        if (a.E != b.E) return a.E < b.E;
        if (a.c != b.c) return a.c < b.c;
        return a.groups < b.groups;
    });
    const int total = (int)found.size();
    for (int k = 0; k < std::min(total, cap); ++k) {
        lbm_dvm_model_t &m = out[k];
        std::memset(&m, 0, sizeof(m));
        m.dim = dim;
        m.V = found[k].V;
        m.E = found[k].E;
        m.n_groups = (int)found[k].groups.size();
        m.c = (double)found[k].c;
        for (int q = 0; q < m.n_groups; ++q) {
            const Vec &g = gens[found[k].groups[q]].g;
            for (int d = 0; d < dim; ++d) m.gen[q * dim + d] = g[d];
            m.w_group[q] = (double)found[k].w[q];
        }
    }
    if (n_out) *n_out = total;
    if (total > cap) return fail(LBM_E_NO_MEMORY, "lbm_dvm_enumerate: more models than cap");
    return LBM_OK;
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
