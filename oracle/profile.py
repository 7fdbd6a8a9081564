"""Oracle: slip velocity and Knudsen-layer analysis of a channel profile.

TEST INFRASTRUCTURE. Only tests, the smoke check and the CPU-baseline leg of the
benchmark may import this module. The product library never calls it and it
shares no code with the product library.

What is computed follows Section VI of the paper (plane Poiseuille flow):

* the slip velocity u_s = u(wall) / u(centre) (Eq. defSlip);
* the parabolic profile u^NS with the same mass flow as u (Eq. uNS) and the
  non-equilibrium (Knudsen-layer) part u^neq = u - u^NS (Eq. uNEQ).

The profile is given at the nodes y_j = (j + 1/2) / ny, j = 0 .. ny-1, of a
channel with walls at y = 0 and y = 1 (half a spacing beyond the first and last
node); z in the paper's notation is y - 1/2 here.

Readings (the paper gives the continuum definitions only):
* u(wall): the quadratic through the three nodes nearest a wall, evaluated on
  the wall, averaged over the two walls;
* u(centre): the middle node for odd ny; for even ny the cubic through the four
  middle nodes evaluated at the centre;
* u^NS: the integral in Eq. uNS and the mass flow are node averages (the
  midpoint rule used for the mass flow, Eq. pf.1). For u^NS to keep that
  discrete mass flow exactly, the continuum factor 3 / (l0/2)^2 = 1 / <z^2>
  becomes 1 / (node average of z^2); the two agree as ny grows.
"""
from __future__ import annotations

import numpy as np


def _lagrange_at(xs, ys, x):
    """Value at x of the polynomial through the points (xs, ys), by the
    Lagrange formula."""
    total = 0.0
    for i, (xi, yi) in enumerate(zip(xs, ys)):
        li = 1.0
        for j, xj in enumerate(xs):
            if j != i:
                li *= (x - xj) / (xi - xj)
        total += li * yi
    return total


def analyse(u):
    """Returns dict(u_wall, u_center, slip, mean, u_ns, u_neq) for a profile
    u[ny] (ny >= 4, or ny = 3)."""
    u = np.asarray(u, dtype=np.float64)
    ny = len(u)
    if ny < 3:
        raise ValueError("need at least three nodes")
    y = (np.arange(ny) + 0.5) / ny
    # wall values: quadratic through the three nearest nodes, at y = 0 and y = 1
    lo = _lagrange_at(y[:3], u[:3], 0.0)
    hi = _lagrange_at(y[-3:], u[-3:], 1.0)
    u_wall = 0.5 * (lo + hi)
    if ny % 2:
        u_center = float(u[ny // 2])
    else:
        if ny < 4:
            raise ValueError("even profiles need at least four nodes")
        k = ny // 2
        u_center = _lagrange_at(y[k - 2:k + 2], u[k - 2:k + 2], 0.5)
    mean = float(np.mean(u))
    z = y - 0.5
    z2 = float(np.mean(z * z))
    u_ns = u_center * (1.0 - (1.0 - mean / u_center) * z * z / z2)
    return dict(u_wall=u_wall, u_center=u_center, slip=u_wall / u_center, mean=mean,
                u_ns=u_ns, u_neq=u - u_ns)
