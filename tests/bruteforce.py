"""Pure-Python dictionary implementation of one channel step, used only to pin
the C oracle on tiny grids (a second, literal re-derivation of the same update).

Populations are a dict {(i, j, velocity tuple): value}. The equilibrium uses
the scalar Hermite recurrence along u (u^n : H^(n)(xi) = |u|^n He_n(u.xi/|u|)),
which is a different formula from the oracle's tensor contraction.
"""
import math


def _dot(a, b):
    return sum(x * y for x, y in zip(a, b))


def equilibrium(w, xi, rho, u, N):
    ue = _dot(u, xi)
    uu = _dot(u, u)
    P = [1.0, ue]
    for n in range(1, N):
        P.append(ue * P[n] - n * uu * P[n - 1])
    return rho * w * sum(P[n] / math.factorial(n) for n in range(N + 1))


def force(w, xi, rho, u, g, Pi):
    D = len(xi)
    gx = _dot(g, xi)
    t = gx + gx * _dot(u, xi) - _dot(u, g)
    s = 0.0
    for i in range(D):
        for j in range(D):
            a2 = Pi[i][j] - (rho if i == j else 0.0)
            h2 = xi[i] * xi[j] - (1.0 if i == j else 0.0)
            s += a2 * (gx * h2 - 2.0 * g[i] * xi[j])
    return rho * w * (t + s / (2.0 * rho))


def _fold(y, ny):
    """Cell-unit coordinate y (walls at 0 and ny) folded back into the channel
    by reflection in the wall it crossed."""
    if y < 0:
        return -y
    if y > ny:
        return 2 * ny - y
    return y


def step(f, vels, weights, c, nx, ny, N, tau, dt, g, alpha=1.0):
    """One stream + collide step of a 2D channel with walls at y (half-way).
    alpha: Maxwell accommodation; the fraction 1 - alpha of each wall value is
    the specularly reflected population, found by following the arriving
    particle back over one step and folding its path at the wall."""
    ws = dict(zip(vels, weights))

    def shape(e):
        return ws[e] * (1.0 - 0.5 * dt * _dot(g, (c * e[0], c * e[1])))

    # wall balance per (wall, element); the element of a crossing is the column
    # of the fluid node it leaves from or arrives at
    A, Dn = {}, {}
    for i in range(nx):
        for j in range(ny):
            for e in vels:
                jd = j + e[1]
                if jd < 0 or jd >= ny:
                    key = (0 if jd < 0 else 1, i)
                    A[key] = A.get(key, 0.0) + f[(i, j, e)]
                js = j - e[1]
                if js < 0 or js >= ny:
                    key = (0 if js < 0 else 1, i)
                    Dn[key] = Dn.get(key, 0.0) + shape(e)
    pre = {}
    for i in range(nx):
        for j in range(ny):
            for e in vels:
                js = j - e[1]
                if 0 <= js < ny:
                    pre[(i, j, e)] = f[((i - e[0]) % nx, js, e)]
                else:
                    key = (0 if js < 0 else 1, i)
                    val = A.get(key, 0.0) / Dn[key] * shape(e)
                    if alpha != 1.0:
                        # start of the folded path: cell centre j + 1/2 moved
                        # back by e_y, reflected in the wall, velocity reversed
                        yc = _fold(j + 0.5 - e[1], ny)
                        src = ((i - e[0]) % nx, int(round(yc - 0.5)), (e[0], -e[1]))
                        val = alpha * val + (1.0 - alpha) * f[src]
                    pre[(i, j, e)] = val
    out = {}
    omega = dt / (tau + 0.5 * dt)
    h = dt / (2.0 * tau)
    for i in range(nx):
        for j in range(ny):
            fb = {e: pre[(i, j, e)] for e in vels}
            rho = sum(fb.values())
            jm = [sum(fb[e] * c * e[d] for e in vels) for d in range(2)]
            u = [(jm[d] + 0.5 * dt * rho * g[d]) / rho for d in range(2)]
            S = [[sum(fb[e] * c * e[a] * c * e[b] for e in vels) for b in range(2)] for a in range(2)]
            # second moment of the generalised equilibrium: rho (I + uu) + tau rho (gu + ug)
            Seq = [[rho * ((1.0 if a == b else 0.0) + u[a] * u[b]) + tau * rho * (g[a] * u[b] + g[b] * u[a])
                    for b in range(2)] for a in range(2)]
            Pi = [[(S[a][b] + h * Seq[a][b]) / (1.0 + h) for b in range(2)] for a in range(2)]
            for e in vels:
                xi = (c * e[0], c * e[1])
                feq = equilibrium(ws[e], xi, rho, u, N) + tau * force(ws[e], xi, rho, u, g, Pi)
                out[(i, j, e)] = fb[e] - omega * (fb[e] - feq)
    return out
