"""Oracle: discrete velocity models (DVMs) from the Hermite null-space construction.

TEST INFRASTRUCTURE. Only tests, the smoke check and the CPU-baseline leg of the
benchmark may import this module. The product library never calls it and it
shares no code with the product library.

What is computed follows Section II of the paper ("Definition of Lattice-Boltzmann
models"):

* tensor Hermite polynomials built by the recurrence H^(n+1) = (xi - d/dxi) H^(n)
  (Eq. defH), kept as exact polynomials with rational coefficients;
* velocity groups S_g generated from one velocity by the lattice reflections,
  all sharing one weight (Eq. wdach);
* the symmetric matrix K(S) of contracted Hermite tensors (Eq. defK), whose null
  space gives the weights, normalised to sum to one (Eq. defQua);
* the lattice speed c enters K(S) through xi = c * e; minimal DVMs exist only
  at discrete c* where K(S) becomes singular (Eq. dimker), and only positive
  weights are accepted.

Restricting K(S) to weight vectors that are constant on groups gives the G x G
matrix K_g(c) = P^T K(S) P. It is positive semi-definite, so its smallest
eigenvalue touches zero at c*; its derivative (Hellmann-Feynman:
n^T K_g'(c) n for the unit eigenvector n) changes sign there and is used as the
root function. Everything after the float64 bracket search runs in mpmath.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field
from fractions import Fraction
from functools import lru_cache

import mpmath as mp
import numpy as np

MP_DPS = 40


# --------------------------------------------------------------------------
# velocity groups (Eq. wdach): reflections of one generator on the lattice's
# symmetry hyperplanes = all signed permutations of its components.
# --------------------------------------------------------------------------
def orbit(gen) -> list[tuple[int, ...]]:
    gen = tuple(int(v) for v in gen)
    d = len(gen)
    out = set()
    for perm in itertools.permutations(range(d)):
        for signs in itertools.product((1, -1), repeat=d):
            out.add(tuple(signs[k] * gen[perm[k]] for k in range(d)))
    return sorted(out)


# --------------------------------------------------------------------------
# tensor Hermite polynomials (Eq. defH) as dicts {exponent tuple: Fraction}
# --------------------------------------------------------------------------
def _xi_minus_d(poly: dict, k: int) -> dict:
    out: dict = {}
    for exp, coef in poly.items():
        up = list(exp)
        up[k] += 1
        up = tuple(up)
        out[up] = out.get(up, 0) + coef
        if exp[k] > 0:
            dn = list(exp)
            dn[k] -= 1
            dn = tuple(dn)
            out[dn] = out.get(dn, 0) - coef * exp[k]
    return {e: c for e, c in out.items() if c != 0}


@lru_cache(maxsize=None)
def hermite_component(index: tuple, dim: int) -> tuple:
    """H^(n)_{i1..in} as a tuple of (exponent, Fraction) pairs, by Eq. defH."""
    if len(index) == 0:
        return (((0,) * dim, Fraction(1)),)
    prev = dict(hermite_component(index[:-1], dim))
    return tuple(sorted(_xi_minus_d(prev, index[-1]).items()))


def eval_poly(poly, x) -> float:
    tot = 0
    for exp, coef in poly:
        term = coef
        for xd, ed in zip(x, exp):
            term = term * xd ** ed
        tot += term
    return tot


def component_multisets(dim: int, m: int):
    """Distinct components of the symmetric rank-m tensor and the number of
    ordered index tuples each one stands for (m!/prod(n_d!))."""
    for ms in itertools.combinations_with_replacement(range(dim), m):
        counts = [ms.count(d) for d in range(dim)]
        mult = math.factorial(m)
        for n in counts:
            mult //= math.factorial(n)
        yield ms, mult


# --------------------------------------------------------------------------
# K(S) restricted to group-constant weights, as polynomials in c
# --------------------------------------------------------------------------
@dataclass
class _System:
    dim: int
    Q: int
    gens: list
    groups: list          # list of orbits
    sizes: list           # V_g
    rows: list            # per row: (mult, coef[g][k]) exact Fractions
    max_deg: int


def _build_system(dim: int, gens, Q: int) -> _System:
    groups = [orbit(g) for g in gens]
    sizes = [len(o) for o in groups]
    rows = []
    for m in range(1, Q + 1):
        for ms, mult in component_multisets(dim, m):
            poly = hermite_component(ms, dim)
            coef = [[Fraction(0)] * (m + 1) for _ in groups]
            for gi, orb in enumerate(groups):
                for exp, cf in poly:
                    deg = sum(exp)
                    s = 0
                    for e in orb:
                        p = 1
                        for ed, xd in zip(exp, e):
                            p *= xd ** ed
                        s += p
                    if s:
                        coef[gi][deg] += cf * s
            if any(any(c != 0 for c in cg) for cg in coef):
                rows.append((mult, coef))
    return _System(dim, Q, [tuple(g) for g in gens], groups, sizes, rows, Q)


def _matrix_f64(sys: _System, cs: np.ndarray) -> np.ndarray:
    """B(c) for an array of c: shape (len(cs), rows, groups), rows scaled by
    sqrt(multiplicity)."""
    R, G = len(sys.rows), len(sys.groups)
    K1 = sys.max_deg + 1
    C = np.zeros((R, G, K1))
    for r, (mult, coef) in enumerate(sys.rows):
        sm = math.sqrt(mult)
        for g in range(G):
            for k, v in enumerate(coef[g]):
                C[r, g, k] = float(v) * sm
    pw = cs[:, None] ** np.arange(K1)[None, :]
    return np.einsum("rgk,nk->nrg", C, pw)


def _scan(sys: _System, c_lo: float, c_hi: float, n: int = 4000):
    cs = np.linspace(c_lo, c_hi, n)
    B = _matrix_f64(sys, cs)
    ratio = np.empty(n)
    for i in range(n):
        M = B[i]
        rn = np.linalg.norm(M, axis=1)
        M = M[rn > 0] / rn[rn > 0, None]
        cn = np.linalg.norm(M, axis=0)
        M = M / np.where(cn > 0, cn, 1.0)[None, :]
        s = np.linalg.svd(M, compute_uv=False)
        ratio[i] = s[-1] / s[0]
    cands = []
    for i in range(1, n - 1):
        if ratio[i] <= ratio[i - 1] and ratio[i] <= ratio[i + 1] and ratio[i] < 1e-2:
            cands.append((cs[i - 1], cs[i], cs[i + 1]))
    return cands


def _mp_rows(sys: _System):
    """Row coefficients converted once to mpmath numbers."""
    out = []
    for mult, coef in sys.rows:
        out.append((mult, [[mp.mpf(cf.numerator) / cf.denominator for cf in cg]
                           for cg in coef]))
    return out


def _mp_Kg(mrows, G, c, rs, cscale):
    """K_g(c) and dK_g/dc in mpmath, rows scaled by rs, columns by cscale."""
    K = [[mp.mpf(0)] * G for _ in range(G)]
    Kp = [[mp.mpf(0)] * G for _ in range(G)]
    for r, (mult, coef) in enumerate(mrows):
        b = []
        bp = []
        for g in range(G):
            cg = coef[g]
            v = mp.mpf(0)
            vp = mp.mpf(0)
            for k in range(len(cg) - 1, -1, -1):      # Horner for p and p'
                vp = vp * c + v
                v = v * c + cg[k]
            b.append(v * cscale[g])
            bp.append(vp * cscale[g])
        wgt = mult * rs[r] ** 2
        if not wgt:
            continue
        for i in range(G):
            wi = wgt * b[i]
            wpi = wgt * bp[i]
            Ki, Kpi = K[i], Kp[i]
            for j in range(G):
                Ki[j] += wi * b[j]
                Kpi[j] += wpi * b[j] + wi * bp[j]
    return mp.matrix(K), mp.matrix(Kp)


def _refine(sys: _System, c0: float, c_left: float, c_right: float):
    mp.mp.dps = MP_DPS
    G = len(sys.groups)
    B0 = _matrix_f64(sys, np.array([c0]))[0]
    rn = np.linalg.norm(B0, axis=1)
    rs = [mp.mpf(1) / mp.mpf(float(x)) if x > 0 else mp.mpf(0) for x in rn]
    # the sqrt(mult) is already inside B0's norm; _mp_Kg multiplies by mult
    rs = [r_ / mp.sqrt(sys.rows[i][0]) if r_ else r_ for i, r_ in enumerate(rs)]
    B0n = B0 / np.where(rn > 0, rn, 1.0)[:, None]
    cn = np.linalg.norm(B0n, axis=0)
    cscale = [mp.mpf(1) / mp.mpf(float(x)) for x in cn]

    mrows = _mp_rows(sys)

    def dlam(c):
        K, Kp = _mp_Kg(mrows, G, c, rs, cscale)
        ev, evec = mp.eigsy(K)
        i = min(range(G), key=lambda k: ev[k])
        n = evec[:, i]
        return (n.T * Kp * n)[0], ev[i], n

    a, b = mp.mpf(c_left), mp.mpf(c_right)
    fa, _, _ = dlam(a)
    fb, _, _ = dlam(b)
    if fa * fb > 0:
        return None
    # Illinois regula falsi on the sign-changing derivative of lambda_min
    side = 0
    c_prev = None
    tol = mp.mpf(10) ** (-(MP_DPS - 8))
    for _ in range(100):
        c = b - fb * (b - a) / (fb - fa)
        fc, lam, n = dlam(c)
        if fc == 0 or (c_prev is not None and abs(c - c_prev) < tol * abs(c)):
            break
        c_prev = c
        if fa * fc < 0:
            b, fb = c, fc
            if side == -1:
                fa /= 2
            side = -1
        else:
            a, fa = c, fc
            if side == 1:
                fb /= 2
            side = 1
    fc, lam, n = dlam(c)
    wbar = [n[g] * cscale[g] for g in range(G)]
    norm = sum(sys.sizes[g] * wbar[g] for g in range(G))
    wbar = [x / norm for x in wbar]
    return c, lam, wbar


@dataclass
class DVM:
    dim: int
    Q: int
    c: float
    gens: list
    group_weights: list           # w_bar_g as floats
    velocities: np.ndarray        # (V, dim) integers e_alpha (xi = c * e)
    weights: np.ndarray           # (V,) float64
    group_of: np.ndarray          # (V,) group index
    c_mp: object = None
    group_weights_mp: list = field(default_factory=list)
    residual: float = 0.0

    @property
    def V(self) -> int:
        return len(self.weights)

    @property
    def xi(self) -> np.ndarray:
        return self.c * self.velocities.astype(np.float64)

    @property
    def energy(self) -> int:
        """Stencil energy E = sum |xi|^2 / (2 c^2) (Section II.B)."""
        return int(sum(int(np.dot(e, e)) for e in self.velocities)) // 2


def make_dvm(dim: int, gens, group_weights, c, Q: int) -> DVM:
    """Expand groups into velocities with the given (printed or solved) weights."""
    vel, w, gi = [], [], []
    for g, gen in enumerate(gens):
        for e in orbit(gen):
            vel.append(e)
            w.append(float(group_weights[g]))
            gi.append(g)
    return DVM(dim, Q, float(c), [tuple(g) for g in gens],
               [float(x) for x in group_weights],
               np.array(vel, dtype=np.int64), np.array(w), np.array(gi))


def _roots_iter(dim, gens, Q, c_lo, c_hi, n_scan):
    sys = _build_system(dim, gens, Q)
    for cl, cm, cr in _scan(sys, c_lo, c_hi, n_scan):
        res = _refine(sys, cm, cl, cr)
        if res is None:
            continue
        c, lam, wbar = res
        if lam > mp.mpf(10) ** (-(MP_DPS // 2)):
            continue
        yield c, wbar, lam


def solve_roots(dim: int, gens, Q: int, c_lo: float, c_hi: float, n_scan: int = 4000):
    """All c in [c_lo, c_hi] at which K(S) has a group-symmetric null vector."""
    return list(_roots_iter(dim, gens, Q, c_lo, c_hi, n_scan))


def solve_dvm(dim: int, gens, Q: int, c_lo: float = 0.2, c_hi: float = 3.0,
              n_scan: int = 4000) -> DVM:
    """Minimal DVM of order Q on the given groups: the smallest c* in range whose
    weights are all positive (only positive weights are admitted)."""
    for c, wbar, lam in _roots_iter(dim, gens, Q, c_lo, c_hi, n_scan):
        if all(x > 0 for x in wbar):
            d = make_dvm(dim, gens, [float(x) for x in wbar], float(c), Q)
            d.c_mp = c
            d.group_weights_mp = wbar
            d.residual = float(lam)
            return d
    raise ValueError(f"no positive-weight root of K(S) in [{c_lo}, {c_hi}]")


# --------------------------------------------------------------------------
# Quadrature checks (Eqs. genQua / orth): Gaussian moments of omega
# --------------------------------------------------------------------------
def gaussian_moment(exps) -> int:
    """Integral of omega(xi) * prod xi_d^a_d over R^D: prod (a_d - 1)!! for even a_d."""
    out = 1
    for a in exps:
        if a % 2:
            return 0
        out *= math.prod(range(a - 1, 0, -2)) if a > 0 else 1
    return out


def quadrature_errors(dvm: DVM, degree: int):
    """Max relative error of sum_alpha w_alpha xi^a against the Gaussian moment
    over all monomials of total degree `degree`."""
    xi = dvm.xi
    worst = 0.0
    for exps in itertools.product(range(degree + 1), repeat=dvm.dim):
        if sum(exps) != degree:
            continue
        q = float(np.sum(dvm.weights * np.prod(xi ** np.array(exps)[None, :], axis=1)))
        ex = gaussian_moment(exps)
        scale = max(1.0, abs(ex))
        worst = max(worst, abs(q - ex) / scale)
    return worst


def quadrature_degree(dvm: DVM, tol: float = 1e-12, max_degree: int = 14) -> int:
    deg = 0
    while deg + 1 <= max_degree and quadrature_errors(dvm, deg + 1) < tol:
        deg += 1
    return deg


# --------------------------------------------------------------------------
# the three channel/duct DVMs and their groups
# --------------------------------------------------------------------------
D2V17_GENS = [(0, 0), (1, 0), (1, 1), (2, 2), (3, 0)]
D2V37_GENS = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2), (3, 0), (3, 1)]
D3V39_GENS = [(0, 0, 0), (1, 0, 0), (1, 1, 1), (2, 0, 0), (2, 2, 0), (3, 0, 0)]

NAMED = {
    "D2V17": (2, D2V17_GENS, 7),
    "D2V37": (2, D2V37_GENS, 9),
    "D3V39": (3, D3V39_GENS, 7),
}


@lru_cache(maxsize=None)
def named_dvm(name: str) -> DVM:
    dim, gens, Q = NAMED[name]
    return solve_dvm(dim, gens, Q)
