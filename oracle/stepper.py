"""Oracle: Python driver of the FP64 C time stepper (lbm_oracle.c).

TEST INFRASTRUCTURE. Only tests, the smoke check and the CPU-baseline leg of the
benchmark may import this module; the product library never does.

Parameters follow Section V of the paper:
  * tau = nu (Eq. nm.11) and Kn = sqrt(pi/2) tau (Eq. nm.13), so tau = Kn sqrt(2/pi);
  * on-lattice streaming xi * dt = e * dx with dx = l0 / L (L nodes across the
    channel, half-way walls), so dt = 1 / (c L) in units l0 = c0 = 1;
  * omega = dt / (tau + dt/2) (Eq. nm.8);
  * the body force is set from the Navier-Stokes no-slip centreline velocity
    u_c = g l0^2 / (8 nu) (Section VI) so that u_c = Ma: g = 8 tau Ma;
  * normalised mass flow m = <u_x> / (4 u_c Kn) (Eq. pf.1), the average taken
    over the channel cross-section (and x).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
_SO = HERE / "liblbm_oracle.so"
_SRC = HERE / "lbm_oracle.c"


def build(force: bool = False) -> Path:
    """Compile the oracle with gcc (plain C99 + OpenMP)."""
    if force or not _SO.exists() or _SO.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = str(_SO) + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, str(_SRC), "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("V", ctypes.c_int), ("N", ctypes.c_int),
                ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("walls_z", ctypes.c_int), ("pad_", ctypes.c_int),
                ("e", ctypes.POINTER(ctypes.c_int)), ("w", ctypes.POINTER(ctypes.c_double)),
                ("c", ctypes.c_double), ("tau", ctypes.c_double), ("dt", ctypes.c_double),
                ("g", ctypes.c_double * 3), ("alpha", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(str(build()))
        P = ctypes.POINTER(_Problem)
        dp = ctypes.POINTER(ctypes.c_double)
        for name, args in {
            "orc_stream": [P, dp, dp], "orc_collide": [P, dp, dp],
            "orc_moments": [P, dp, dp, dp], "orc_init": [P, dp, dp, dp],
            "orc_run": [P, dp, dp, ctypes.c_long, ctypes.c_int],
            "orc_wall_balance": [P, dp, dp, dp],
            "orc_equilibrium": [P, ctypes.c_double, dp, dp],
            "orc_force": [P, ctypes.c_double, dp, dp, dp],
            "orc_collide_node": [P, dp, dp], "orc_max_threads": [],
        }.items():
            fn = getattr(_lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def tau_from_kn(kn: float) -> float:
    return kn * math.sqrt(2.0 / math.pi)


class Params:
    """Per-solve scalars (a0): tau, dt, omega, g."""

    def __init__(self, c: float, L: int, kn: float, ma: float | None = None,
                 g: tuple | None = None):
        self.kn = kn
        self.tau = tau_from_kn(kn)
        self.dt = 1.0 / (c * L)
        self.omega = self.dt / (self.tau + 0.5 * self.dt)
        if g is None:
            ma = 1e-3 if ma is None else ma
            g = (8.0 * self.tau * ma, 0.0, 0.0)
        self.g = tuple(float(x) for x in g) + (0.0,) * (3 - len(g))
        # centreline speed used to normalise the mass flow (pf.1, pf.2)
        self.u_c = self.g[0] / (8.0 * self.tau) if self.g[0] != 0 else (ma or 1e-3)


class OracleSolver:
    """FP64 oracle channel (2D, walls at y) or duct (3D, walls at y and z)."""

    def __init__(self, dvm, nx: int, ny: int, nz: int = 1, kn: float = 0.1,
                 ma: float | None = 1e-3, N: int = 3, walls_z: bool = False,
                 g: tuple | None = None, alpha: float = 1.0):
        """alpha: Maxwell accommodation (1 = the paper's fully diffuse wall);
        below 1 only for channels (walls normal to y)."""
        if not 0.0 <= alpha <= 1.0:
            raise ValueError("accommodation must lie in [0, 1]")
        if alpha != 1.0 and (dvm.dim != 2 or walls_z):
            raise ValueError("accommodation below 1: channels (walls normal to y) only")
        self.dvm = dvm
        self.dim = dvm.dim
        self.nx, self.ny, self.nz = nx, ny, (nz if dvm.dim == 3 else 1)
        self.walls_z = bool(walls_z) and dvm.dim == 3
        self.N = N
        self.params = Params(dvm.c, ny, kn, ma, g)
        V = dvm.V
        e3 = np.zeros((V, 3), dtype=np.int32)
        e3[:, : dvm.dim] = dvm.velocities
        self._e = np.ascontiguousarray(e3)
        self._w = np.ascontiguousarray(dvm.weights, dtype=np.float64)
        p = _Problem()
        p.dim, p.V, p.N = dvm.dim, V, N
        p.nx, p.ny, p.nz = self.nx, self.ny, self.nz
        p.walls_z = int(self.walls_z)
        p.e = self._e.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        p.w = _dp(self._w)
        p.c, p.tau, p.dt = dvm.c, self.params.tau, self.params.dt
        for d in range(3):
            p.g[d] = self.params.g[d]
        p.alpha = float(alpha)
        self._p = p
        self.nodes = self.nx * self.ny * self.nz
        self.f = np.zeros((self.nodes, V))
        self._tmp = np.zeros_like(self.f)
        self.steps = 0

    # -- state --------------------------------------------------------------
    def init(self, rho=None, u=None):
        """Post-collision state := f^(0)(rho, u) (rest state rho w by default)."""
        rho = np.ones(self.nodes) if rho is None else np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        up = None
        if u is not None:
            up = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(self.nodes, 3))
        lib().orc_init(ctypes.byref(self._p), _dp(rho), _dp(up) if up is not None else None, _dp(self.f))
        self.steps = 0
        return self

    def run(self, nsteps: int, nthreads: int = 0):
        rc = lib().orc_run(ctypes.byref(self._p), _dp(self.f), _dp(self._tmp), int(nsteps), int(nthreads))
        if rc:
            raise MemoryError("oracle run failed")
        self.steps += nsteps
        return self

    def stream(self, fpost=None):
        fpost = self.f if fpost is None else fpost
        out = np.zeros_like(self.f)
        lib().orc_stream(ctypes.byref(self._p), _dp(fpost), _dp(out))
        return out

    def collide(self, fpre):
        out = np.zeros_like(self.f)
        lib().orc_collide(ctypes.byref(self._p), _dp(np.ascontiguousarray(fpre)), _dp(out))
        return out

    def moments(self, fpre):
        rho = np.zeros(self.nodes)
        u = np.zeros((self.nodes, 3))
        lib().orc_moments(ctypes.byref(self._p), _dp(np.ascontiguousarray(fpre)), _dp(rho), _dp(u))
        return rho, u

    def wall_balance(self, fpost=None):
        fpost = self.f if fpost is None else fpost
        ne = max(self.nx * self.nz, self.nx * self.ny)
        A = np.zeros(4 * ne)
        D = np.zeros(4 * ne)
        lib().orc_wall_balance(ctypes.byref(self._p), _dp(fpost), _dp(A), _dp(D))
        return A.reshape(4, ne), D.reshape(4, ne)

    # -- observables ----------------------------------------------------------
    def observe(self):
        """Moments of the state after streaming the current post-collision
        populations (the pre-collision state of the next step)."""
        rho, u = self.moments(self.stream())
        shape = (self.nz, self.ny, self.nx) if self.dim == 3 else (self.ny, self.nx)
        ux_mean = float(np.mean(u[:, 0]))
        return dict(rho=rho.reshape(shape), u=u.reshape(shape + (3,)),
                    mdot=ux_mean / (4.0 * self.params.u_c * self.params.kn),
                    mass=float(np.sum(self.f)))

    def populations(self):
        """Post-collision populations as [alpha][z][y][x] (2D: [alpha][y][x])."""
        shape = (self.nz, self.ny, self.nx) if self.dim == 3 else (self.ny, self.nx)
        return np.moveaxis(self.f.reshape(shape + (self.dvm.V,)), -1, 0).copy()

    # -- single-node helpers ----------------------------------------------------
    def equilibrium(self, rho, u):
        out = np.zeros(self.dvm.V)
        uu = np.zeros(3)
        uu[: len(u)] = u
        lib().orc_equilibrium(ctypes.byref(self._p), float(rho), _dp(uu), _dp(out))
        return out

    def force(self, rho, u, Pi=None):
        out = np.zeros(self.dvm.V)
        uu = np.zeros(3)
        uu[: len(u)] = u
        P = None
        if Pi is not None:
            P = np.zeros((3, 3))
            Pi = np.asarray(Pi, dtype=np.float64)
            P[: Pi.shape[0], : Pi.shape[1]] = Pi
            P = np.ascontiguousarray(P)
        lib().orc_force(ctypes.byref(self._p), float(rho), _dp(uu), _dp(P) if P is not None else None, _dp(out))
        return out

    def collide_node(self, fb):
        fb = np.ascontiguousarray(fb, dtype=np.float64)
        out = np.zeros(self.dvm.V)
        lib().orc_collide_node(ctypes.byref(self._p), _dp(fb), _dp(out))
        return out


def max_threads() -> int:
    return lib().orc_max_threads()
