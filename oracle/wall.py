"""Oracle: equilibrium wall moments of a DVM and their errors.

TEST INFRASTRUCTURE. Only tests, the smoke check and the CPU-baseline leg of the
benchmark may import this module. The product library never calls it and it
shares no code with the product library.

What is computed follows Section IV of the paper (diffuse Maxwell boundary
condition and wall moments):

* the exact half-space moments W of the weight function omega (Eq. defW), by
  the closed form of Eq. Wscalar with Euler's Gamma function;
* their quadrature over the velocities pointing away from the wall into the
  fluid (Eq. wallQuad);
* the relative errors sigma of each moment and their e^-n weighted mean
  sigma_Sigma (Eqs. wallError, sigmaSigma) over the non-trivial components of
  Eq. nontriv, in the order of Eqs. defT / defb;
* the wall accuracy index Lambda_index (Eq. defbin) and order Lambda
  (Eq. defLambda).

Coordinates: z is the wall normal (n = e_z, pointing into the fluid), x and y
are tangential; a 2D model has only x and z (the y exponent is 0).

Readings where the paper is ambiguous:
* sign of sigma: the tables print (W^DVM - W) / W, the opposite of the sign in
  Eq. wallError; the tables' sign is used;
* sigma_Sigma runs over the L non-trivial components of Eq. nontriv (each
  multiset of exponents once), with weight e^-n for a moment of rank n;
* "a constraint holds" and "sigma = 0" are decided to a relative 1e-10, far
  above the rounding of the weights and far below any printed error.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

EXACT_TOL = 1e-10


def exact_moment(mx: int, my: int, mz: int, dim: int = 3) -> float:
    """Eq. Wscalar: integral over the half space xi_z > 0 of omega xi_x^mx
    xi_y^my xi_z^mz, omega the unit-variance Gaussian of dimension dim. In 2D
    the y integral is absent (my must be 0)."""
    if dim == 2:
        if my:
            raise ValueError("2D moments have no y component")
        # one full-line Gaussian integral in x and one half-line in z
        return (math.sqrt(2.0) ** (mx + mz) / (4.0 * math.pi)) * (1 + (-1) ** mx) * \
            math.gamma((mx + 1) / 2.0) * math.gamma((mz + 1) / 2.0)
    return (math.sqrt(2.0) ** (mx + my + mz) / (8.0 * math.sqrt(math.pi) ** 3)) * \
        (1 + (-1) ** mx) * (1 + (-1) ** my) * \
        math.gamma((mx + 1) / 2.0) * math.gamma((my + 1) / 2.0) * math.gamma((mz + 1) / 2.0)


def _axes(dim: int, normal: int):
    """Indices of (x, y, z) in a velocity vector: z = normal, x and y the
    remaining axes in increasing order (y = None in 2D)."""
    rest = [a for a in range(dim) if a != normal]
    return rest[0], (rest[1] if dim == 3 else None), normal


def dvm_moment(xi: np.ndarray, w: np.ndarray, mx: int, my: int, mz: int, normal: int) -> float:
    """Eq. wallQuad: sum over velocities with n.xi > 0 of w xi_x^mx xi_y^my xi_z^mz."""
    dim = xi.shape[1]
    ax, ay, az = _axes(dim, normal)
    sel = xi[:, az] > 0
    v = w[sel] * xi[sel, ax] ** mx * xi[sel, az] ** mz
    if ay is not None:
        v = v * xi[sel, ay] ** my
    return float(np.sum(v))


def nontrivial_components(Q: int, dim: int = 3):
    """Eq. nontriv in the order of Eqs. defT / defb: increasing rank n, then
    decreasing m_z, then decreasing m_x. m_x, m_y even with m_y <= m_x (m_y = 0
    in 2D), m_z = 0 or odd, m_x + m_y + m_z <= Q."""
    out = []
    for n in range(Q + 1):
        for mz in range(n, -1, -1):
            if not (mz == 0 or mz % 2 == 1):
                continue
            for mx in range(n - mz, -1, -1):
                my = n - mz - mx
                if mx % 2 or my % 2 or my > mx:
                    continue
                if dim == 2 and my:
                    continue
                out.append((mx, my, mz))
    return out


def wall_errors(dvm, normal: int | None = None, Q: int | None = None):
    """Wall moments and errors of a DVM (oracle DVM object: velocities, weights,
    c, dim, Q). Returns a dict with the component list, W, W^DVM, sigma,
    sigma_Sigma, Lambda_index and Lambda."""
    dim = dvm.dim
    Q = dvm.Q if Q is None else Q
    normal = dim - 1 if normal is None else normal
    xi = dvm.c * np.asarray(dvm.velocities, dtype=np.float64)
    w = np.asarray(dvm.weights, dtype=np.float64)
    comps = nontrivial_components(Q, dim)
    W = [exact_moment(mx, my, mz, dim) for (mx, my, mz) in comps]
    Wd = [dvm_moment(xi, w, mx, my, mz, normal) for (mx, my, mz) in comps]
    sigma = [(b - a) / a for a, b in zip(W, Wd)]
    num = sum(abs(s) * math.exp(-sum(c)) for s, c in zip(sigma, comps))
    den = sum(math.exp(-sum(c)) for c in comps)
    index = sum(1 << k for k, s in enumerate(sigma) if abs(s) <= EXACT_TOL)
    return dict(components=comps, W=W, W_dvm=Wd, sigma=sigma, sigma_sigma=num / den,
                lambda_index=index, lambda_order=wall_order(dvm, normal, Q))


def wall_order(dvm, normal: int | None = None, Q: int | None = None) -> int:
    """Eq. defLambda: the largest Lambda <= Q such that every wall moment of
    rank n <= Lambda (every exponent triple, trivial ones included) is exact;
    -1 if the zeroth one is not. A moment whose exact value vanishes counts as
    exact when its quadrature vanishes to EXACT_TOL times the moment's scale."""
    dim = dvm.dim
    Q = dvm.Q if Q is None else Q
    normal = dim - 1 if normal is None else normal
    xi = dvm.c * np.asarray(dvm.velocities, dtype=np.float64)
    w = np.asarray(dvm.weights, dtype=np.float64)
    order = -1
    for n in range(Q + 1):
        ok = True
        for mx, my, mz in _triples(n, dim):
            a = exact_moment(mx, my, mz, dim)
            b = dvm_moment(xi, w, mx, my, mz, normal)
            scale = abs(a) if a != 0 else _abs_moment(xi, w, mx, my, mz, normal)
            if abs(b - a) > EXACT_TOL * max(scale, 1e-300):
                ok = False
                break
        if not ok:
            break
        order = n
    return order


def _triples(n: int, dim: int):
    if dim == 2:
        return [(mx, 0, n - mx) for mx in range(n + 1)]
    return [(mx, my, n - mx - my) for mx, my in itertools.product(range(n + 1), repeat=2)
            if mx + my <= n]


def _abs_moment(xi, w, mx, my, mz, normal):
    dim = xi.shape[1]
    ax, ay, az = _axes(dim, normal)
    sel = xi[:, az] > 0
    v = w[sel] * np.abs(xi[sel, ax]) ** mx * np.abs(xi[sel, az]) ** mz
    if ay is not None:
        v = v * np.abs(xi[sel, ay]) ** my
    return float(np.sum(v))
