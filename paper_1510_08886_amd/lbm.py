"""Python binding of liblbmdvm.so (ctypes): argument marshalling only.

PyTorch supplies device memory (tensors) and the HIP stream; every step of the
lattice update runs in the library's HIP kernels. There is no CPU fallback: if
the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from pathlib import Path

import numpy as np

PKG = Path(__file__).resolve().parent
LIB_PATH = PKG / "liblbmdvm.so"

LBM_OK = 0
ERRORS = {-1: "LBM_E_INVALID", -2: "LBM_E_UNSUPPORTED", -3: "LBM_E_NO_MEMORY",
          -4: "LBM_E_QUADRATURE", -5: "LBM_E_DEVICE", -6: "LBM_E_NOT_CONVERGED"}
STORAGE = {"f64": 0, "f32": 1, "f16dev": 2, "f32raw": 3}

# Velocity groups of the three models used for channels and ducts: generators,
# dimension, quadrature order, Hermite order of the equilibrium.
NAMED_DVMS = {
    "D2V17": dict(dim=2, gens=[(0, 0), (1, 0), (1, 1), (2, 2), (3, 0)], Q=7, N=3),
    "D2V37": dict(dim=2, gens=[(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2), (3, 0), (3, 1)],
                  Q=9, N=4),
    "D3V39": dict(dim=3, gens=[(0, 0, 0), (1, 0, 0), (1, 1, 1), (2, 0, 0), (2, 2, 0), (3, 0, 0)],
                  Q=7, N=3),
}


class LbmError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {ERRORS.get(code, code)}: {msg}")
        self.code = code


class ProblemC(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("nz", ctypes.c_int), ("kn", ctypes.c_double), ("ma", ctypes.c_double),
                ("g_set", ctypes.c_int), ("g", ctypes.c_double * 3),
                ("hermite_order", ctypes.c_int), ("accommodation", ctypes.c_double),
                ("rho0", ctypes.c_double), ("storage", ctypes.c_int)]


class ParamsC(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("dt", ctypes.c_double), ("omega", ctypes.c_double),
                ("g", ctypes.c_double * 3), ("u_c", ctypes.c_double),
                ("mdot_scale", ctypes.c_double), ("V", ctypes.c_int), ("halo", ctypes.c_int)]


_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int)
_I32P = ctypes.POINTER(ctypes.c_int32)
_I64 = ctypes.c_int64
_SZP = ctypes.POINTER(ctypes.c_size_t)

SIGNATURES = {
    "lbm_last_error": ([], ctypes.c_char_p),
    "lbm_dvm_solve": ([_I, _I, _I32P, _I, _D, _D, _DP, _DP, _IP], _I),
    "lbm_dvm_create": ([_I, _I, _I32P, _DP, _D, _I, ctypes.POINTER(_P)], _I),
    "lbm_dvm_destroy": ([_P], _I),
    "lbm_dvm_info": ([_P, _IP, _I32P, _DP, _DP], _I),
    "lbm_params": ([_P, ctypes.POINTER(ProblemC), ctypes.POINTER(ParamsC)], _I),
    "lbm_state_bytes": ([_P, ctypes.POINTER(ProblemC), _SZP, _SZP], _I),
    "lbm_solver_create": ([_P, ctypes.POINTER(ProblemC), _P, _P, _P, ctypes.c_size_t, _P,
                           ctypes.POINTER(_P)], _I),
    "lbm_solver_destroy": ([_P], _I),
    "lbm_init_equilibrium": ([_P, _P, _P], _I),
    "lbm_run": ([_P, _I64], _I),
    "lbm_run_to_tol": ([_P, _D, _I, _I64, ctypes.POINTER(_I64), _DP], _I),
    "lbm_observe": ([_P, _P, _P, _DP, _DP], _I),
    "lbm_export_populations": ([_P, _P], _I),
    "lbm_import_populations": ([_P, _P], _I),
    "lbm_solver_steps": ([_P, ctypes.POINTER(_I64)], _I),
}


def lib():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1510_08886_amd.build` (no CPU fallback exists)")
        _lib = ctypes.CDLL(str(LIB_PATH))
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(_lib, name, None)
            if fn is None:
                continue
            fn.argtypes = args
            fn.restype = res
    return _lib


def check(rc: int, where: str):
    if rc != LBM_OK:
        raise LbmError(rc, where, lib().lbm_last_error().decode())


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_I32P)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_DP)


class Dvm:
    """A velocity set with weights, owned by the library."""

    def __init__(self, dim: int, gens, weights, c: float, Q: int):
        g, gp = _i32(np.asarray(gens).reshape(-1))
        w, wp = _f64(weights)
        h = _P()
        check(lib().lbm_dvm_create(dim, len(gens), gp, wp, float(c), Q, ctypes.byref(h)),
              "lbm_dvm_create")
        self._h = h
        self.dim, self.Q, self.gens = dim, Q, [tuple(x) for x in gens]
        V = ctypes.c_int()
        check(lib().lbm_dvm_info(h, ctypes.byref(V), None, None, None), "lbm_dvm_info")
        self.V = V.value
        vel = np.zeros(self.V * dim, dtype=np.int32)
        wv = np.zeros(self.V)
        cc = ctypes.c_double()
        check(lib().lbm_dvm_info(h, None, vel.ctypes.data_as(_I32P), wv.ctypes.data_as(_DP),
                                 ctypes.byref(cc)), "lbm_dvm_info")
        self.velocities = vel.reshape(self.V, dim)
        self.weights = wv
        self.c = cc.value

    @staticmethod
    def solve_weights(dim: int, gens, Q: int, c_lo: float = 0.2, c_hi: float = 3.0):
        g, gp = _i32(np.asarray(gens).reshape(-1))
        c = ctypes.c_double()
        w = np.zeros(len(gens))
        V = ctypes.c_int()
        check(lib().lbm_dvm_solve(dim, len(gens), gp, Q, c_lo, c_hi, ctypes.byref(c),
                                  w.ctypes.data_as(_DP), ctypes.byref(V)), "lbm_dvm_solve")
        return c.value, w, V.value

    @classmethod
    def solve(cls, dim: int, gens, Q: int, c_lo: float = 0.2, c_hi: float = 3.0) -> "Dvm":
        c, w, _ = cls.solve_weights(dim, gens, Q, c_lo, c_hi)
        return cls(dim, gens, w, c, Q)

    @classmethod
    def named(cls, name: str) -> "Dvm":
        spec = NAMED_DVMS[name]
        d = cls.solve(spec["dim"], spec["gens"], spec["Q"])
        d.name = name
        d.default_N = spec["N"]
        return d

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.lbm_dvm_destroy(h)
            self._h = None


@dataclass
class Problem:
    dim: int = 2
    nx: int = 1
    ny: int = 40
    nz: int = 1
    kn: float = 0.1
    ma: float = 1e-3
    g: tuple | None = None
    hermite_order: int = 3
    accommodation: float = 1.0
    rho0: float = 1.0
    storage: str = "f64"

    def to_c(self) -> ProblemC:
        p = ProblemC()
        p.dim, p.nx, p.ny, p.nz = self.dim, self.nx, self.ny, self.nz if self.dim == 3 else 1
        p.kn, p.ma = self.kn, self.ma
        if self.g is not None:
            p.g_set = 1
            for k, v in enumerate(tuple(self.g) + (0.0,) * (3 - len(self.g))):
                p.g[k] = v
        p.hermite_order = self.hermite_order
        p.accommodation = self.accommodation
        p.rho0 = self.rho0
        p.storage = STORAGE[self.storage]
        return p


def params(dvm: Dvm, prob: Problem) -> ParamsC:
    out = ParamsC()
    pc = prob.to_c()
    check(lib().lbm_params(dvm._h, ctypes.byref(pc), ctypes.byref(out)), "lbm_params")
    return out


def state_bytes(dvm: Dvm, prob: Problem):
    pc = prob.to_c()
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    check(lib().lbm_state_bytes(dvm._h, ctypes.byref(pc), ctypes.byref(a), ctypes.byref(b)),
          "lbm_state_bytes")
    return a.value, b.value


def _ptr(t) -> int:
    return t.data_ptr()


class Solver:
    """One channel / duct solve on caller-owned torch device buffers."""

    def __init__(self, dvm: Dvm, prob: Problem, device: str = "cuda", stream=None):
        import torch

        self.torch = torch
        self.dvm, self.prob = dvm, prob
        self.device = torch.device(device)
        pop_b, scr_b = state_bytes(dvm, prob)
        # 256-byte aligned allocations from torch's allocator
        self.pop_a = torch.empty(pop_b, dtype=torch.uint8, device=self.device)
        self.pop_b = torch.empty(pop_b, dtype=torch.uint8, device=self.device)
        self.scratch = torch.empty(scr_b, dtype=torch.uint8, device=self.device)
        for t in (self.pop_a, self.pop_b, self.scratch):
            if t.data_ptr() % 256:
                raise RuntimeError("device allocation is not 256-byte aligned")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.params = params(dvm, prob)
        self.nodes = prob.nx * prob.ny * (prob.nz if prob.dim == 3 else 1)
        self.shape = ((prob.nz, prob.ny, prob.nx) if prob.dim == 3 else (prob.ny, prob.nx))
        pc = prob.to_c()
        h = _P()
        check(lib().lbm_solver_create(dvm._h, ctypes.byref(pc), _ptr(self.pop_a),
                                      _ptr(self.pop_b), _ptr(self.scratch), scr_b,
                                      ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
              "lbm_solver_create")
        self._h = h

    def init(self, rho=None, u=None):
        torch = self.torch
        r = None if rho is None else rho.to(self.device, torch.float64).contiguous().reshape(-1)
        v = None if u is None else u.to(self.device, torch.float64).contiguous().reshape(-1)
        self._keep = (r, v)
        check(lib().lbm_init_equilibrium(self._h, _ptr(r) if r is not None else None,
                                         _ptr(v) if v is not None else None),
              "lbm_init_equilibrium")
        return self

    def run(self, nsteps: int):
        check(lib().lbm_run(self._h, int(nsteps)), "lbm_run")
        return self

    def run_to_tol(self, tol: float = 1e-8, check_every: int = 100, max_steps: int = 10**7):
        steps = ctypes.c_int64()
        md = ctypes.c_double()
        rc = lib().lbm_run_to_tol(self._h, tol, check_every, max_steps, ctypes.byref(steps),
                                  ctypes.byref(md))
        if rc not in (LBM_OK, -6):
            check(rc, "lbm_run_to_tol")
        return dict(steps=steps.value, mdot=md.value, converged=(rc == LBM_OK))

    def observe(self):
        torch = self.torch
        rho = torch.empty(self.nodes, dtype=torch.float64, device=self.device)
        u = torch.empty(self.nodes * 3, dtype=torch.float64, device=self.device)
        md, mass = ctypes.c_double(), ctypes.c_double()
        check(lib().lbm_observe(self._h, _ptr(rho), _ptr(u), ctypes.byref(md), ctypes.byref(mass)),
              "lbm_observe")
        return dict(rho=rho.reshape(self.shape), u=u.reshape(self.shape + (3,)),
                    mdot=md.value, mass=mass.value)

    def mdot(self) -> float:
        md = ctypes.c_double()
        check(lib().lbm_observe(self._h, None, None, ctypes.byref(md), None), "lbm_observe")
        return md.value

    def export(self):
        torch = self.torch
        out = torch.empty(self.dvm.V * self.nodes, dtype=torch.float64, device=self.device)
        check(lib().lbm_export_populations(self._h, _ptr(out)), "lbm_export_populations")
        return out.reshape((self.dvm.V,) + self.shape)

    def import_(self, pops):
        torch = self.torch
        p = pops.to(self.device, torch.float64).contiguous().reshape(-1)
        self._keep = (p,)
        check(lib().lbm_import_populations(self._h, _ptr(p)), "lbm_import_populations")
        return self

    @property
    def steps(self) -> int:
        s = ctypes.c_int64()
        check(lib().lbm_solver_steps(self._h, ctypes.byref(s)), "lbm_solver_steps")
        return s.value

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            lib().lbm_solver_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
