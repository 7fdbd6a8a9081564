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
LBM_E_INVALID = -1
LBM_E_UNSUPPORTED = -2
LBM_E_NO_MEMORY = -3
LBM_E_QUADRATURE = -4
LBM_E_DEVICE = -5
LBM_E_NOT_CONVERGED = -6
ERRORS = {-1: "LBM_E_INVALID", -2: "LBM_E_UNSUPPORTED", -3: "LBM_E_NO_MEMORY",
          -4: "LBM_E_QUADRATURE", -5: "LBM_E_DEVICE", -6: "LBM_E_NOT_CONVERGED"}
STORAGE = {"f64": 0, "f32": 1, "f16dev": 2, "f32raw": 3, "f32sr": 4}
LAYOUT = {"auto": 0, "in_place": 1, "ping_pong": 2}

# Velocity groups of the three models used for channels and ducts: generators,
# dimension, quadrature order, Hermite order of the equilibrium.
NAMED_DVMS = {
    "D2V17": dict(dim=2, gens=[(0, 0), (1, 0), (1, 1), (2, 2), (3, 0)], Q=7, N=3),
    "D2V37": dict(dim=2, gens=[(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2), (3, 0), (3, 1)],
                  Q=9, N=4),
    "D3V39": dict(dim=3, gens=[(0, 0, 0), (1, 0, 0), (1, 1, 1), (2, 0, 0), (2, 2, 0), (3, 0, 0)],
                  Q=7, N=3),
    # scattering stencils (no velocity parallel to a wall)
    "D2V32": dict(dim=2, gens=[(1, 1), (2, 2), (5, 1), (6, 4), (12, 3)], Q=7, N=4),
    "D3V96": dict(dim=3, gens=[(1, 1, 1), (3, 3, 3), (3, 1, 1), (4, 4, 4), (7, 1, 1), (6, 6, 1)],
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
                ("rho0", ctypes.c_double), ("storage", ctypes.c_int), ("layout", ctypes.c_int)]


class ParamsC(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("dt", ctypes.c_double), ("omega", ctypes.c_double),
                ("g", ctypes.c_double * 3), ("u_c", ctypes.c_double),
                ("mdot_scale", ctypes.c_double), ("V", ctypes.c_int), ("halo", ctypes.c_int)]


class ResultC(ctypes.Structure):
    _fields_ = [("req_id", ctypes.c_uint64), ("status", ctypes.c_int), ("ny", ctypes.c_int),
                ("steps", ctypes.c_int64), ("mdot", ctypes.c_double), ("kn", ctypes.c_double)]


class WallReportC(ctypes.Structure):
    _fields_ = [("n_components", ctypes.c_int), ("lambda_order", ctypes.c_int),
                ("lambda_index", ctypes.c_uint64), ("sigma_sigma", ctypes.c_double)]


MAX_GROUPS = 16


class DvmModelC(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("V", ctypes.c_int), ("E", ctypes.c_int),
                ("n_groups", ctypes.c_int), ("gen", ctypes.c_int32 * (MAX_GROUPS * 3)),
                ("c", ctypes.c_double), ("w_group", ctypes.c_double * MAX_GROUPS)]


class ProfileStatsC(ctypes.Structure):
    _fields_ = [("u_center", ctypes.c_double), ("u_wall", ctypes.c_double),
                ("slip", ctypes.c_double), ("mean", ctypes.c_double)]


class BatchTuningC(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_int), ("slots_per_cu", ctypes.c_int), ("order", ctypes.c_int),
                ("trials", ctypes.c_int), ("trial_ms", ctypes.c_float)]


BATCH_ORDERS = {1: "longest_first", 2: "submit"}


class BatchStatsC(ctypes.Structure):
    _fields_ = [("active", ctypes.c_int), ("queued", ctypes.c_int), ("done", ctypes.c_int),
                ("threads", ctypes.c_int), ("quantum", ctypes.c_int), ("slots_per_cu", ctypes.c_int),
                ("order", ctypes.c_int), ("graph_replays", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("pool_used", ctypes.c_size_t), ("pool_free", ctypes.c_size_t)]


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
    "lbm_profile_analysis": ([_DP, _I, ctypes.POINTER(ProfileStatsC), _DP, _DP], _I),
    "lbm_dvm_wall_errors": ([_P, _I, _I, _I32P, _DP, _DP, _DP, ctypes.POINTER(WallReportC)], _I),
    "lbm_params": ([_P, ctypes.POINTER(ProblemC), ctypes.POINTER(ParamsC)], _I),
    "lbm_state_bytes": ([_P, ctypes.POINTER(ProblemC), _SZP, _SZP], _I),
    "lbm_solver_create": ([_P, ctypes.POINTER(ProblemC), _P, _P, _P, ctypes.c_size_t, _P,
                           ctypes.POINTER(_P)], _I),
    "lbm_solver_destroy": ([_P], _I),
    "lbm_solver_create_static": ([_P, ctypes.POINTER(ProblemC), _P, _P, ctypes.POINTER(_P)], _I),
    "lbm_init_equilibrium": ([_P, _P, _P], _I),
    "lbm_run": ([_P, _I64], _I),
    "lbm_run_to_tol": ([_P, _D, _I, _I64, ctypes.POINTER(_I64), _DP], _I),
    "lbm_observe": ([_P, _P, _P, _DP, _DP], _I),
    "lbm_export_populations": ([_P, _P], _I),
    "lbm_import_populations": ([_P, _P], _I),
    "lbm_solver_steps": ([_P, ctypes.POINTER(_I64)], _I),
    "lbm_solver_set_graph_steps": ([_P, _I], _I),
    "lbm_solver_set_pair_steps": ([_P, _I, _I], _I),
    "lbm_solver_set_resident_steps": ([_P, _I], _I),
    "lbm_batch_create": ([_I, _I, _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)], _I),
    "lbm_batch_destroy": ([_P], _I),
    "lbm_batch_submit": ([_P, _P, ctypes.POINTER(ProblemC), _D, _I, _I64, ctypes.c_uint64], _I),
    "lbm_batch_poll": ([_P, ctypes.POINTER(ResultC), _I, _IP], _I),
    "lbm_batch_drain": ([_P, ctypes.POINTER(ResultC), _I, _IP], _I),
    "lbm_batch_run_persistent": ([_P, ctypes.POINTER(ResultC), _I, _IP], _I),
    "lbm_time_launches": ([_P, _P, _I, _I, _I, _P], _I),
    "lbm_batch_tune": ([_P, _I, _I, _I, _I], _I),
    "lbm_batch_autotune": ([_P, _I, _P], _I),
    "lbm_batch_stats": ([_P, ctypes.POINTER(BatchStatsC)], _I),
    "lbm_stream_copy": ([_P, _P, ctypes.c_size_t, _P], _I),
    "lbm_dvm_enumerate": ([_I, _I, _I, _I, _I, _P, _I, _IP], _I),
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


def profile_analysis(u) -> dict:
    """Slip velocity and Knudsen-layer split of a channel profile u[ny] (host
    values, e.g. the x-average of Solver.observe()["u"][..., 0])."""
    u = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(-1))
    ny = len(u)
    st = ProfileStatsC()
    ns, neq = np.zeros(ny), np.zeros(ny)
    check(lib().lbm_profile_analysis(u.ctypes.data_as(_DP), ny, ctypes.byref(st),
                                     ns.ctypes.data_as(_DP), neq.ctypes.data_as(_DP)),
          "lbm_profile_analysis")
    return dict(u_center=st.u_center, u_wall=st.u_wall, slip=st.slip, mean=st.mean, u_ns=ns,
                u_neq=neq)


def stream_copy(src, dst, stream=None):
    """Plain streaming copy between two equally sized contiguous device
    tensors (a bandwidth reference, not part of the method), asynchronous on
    `stream` (default: torch's current stream)."""
    import torch
    if src.numel() * src.element_size() != dst.numel() * dst.element_size():
        raise ValueError("src and dst differ in size")
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("need contiguous device tensors")
    st = stream if stream is not None else torch.cuda.current_stream(src.device)
    check(lib().lbm_stream_copy(_P(src.data_ptr()), _P(dst.data_ptr()),
                                src.numel() * src.element_size(), _P(st.cuda_stream)),
          "lbm_stream_copy")


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

    def wall_errors(self, normal_axis: int | None = None) -> dict:
        """Equilibrium wall moments and their errors (lbm_dvm_wall_errors)."""
        ax = self.dim - 1 if normal_axis is None else int(normal_axis)
        rep = WallReportC()
        check(lib().lbm_dvm_wall_errors(self._h, ax, 0, None, None, None, None, ctypes.byref(rep)),
              "lbm_dvm_wall_errors")
        L = rep.n_components
        ex = np.zeros(3 * L, dtype=np.int32)
        we, wd, sg = np.zeros(L), np.zeros(L), np.zeros(L)
        check(lib().lbm_dvm_wall_errors(self._h, ax, L, ex.ctypes.data_as(_I32P),
                                        we.ctypes.data_as(_DP), wd.ctypes.data_as(_DP),
                                        sg.ctypes.data_as(_DP), ctypes.byref(rep)),
              "lbm_dvm_wall_errors")
        return dict(components=[tuple(int(v) for v in ex[3 * k:3 * k + 3]) for k in range(L)],
                    W=we, W_dvm=wd, sigma=sg, sigma_sigma=rep.sigma_sigma,
                    lambda_index=int(rep.lambda_index), lambda_order=rep.lambda_order)

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
    layout: str = "auto"

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
        p.layout = LAYOUT[self.layout]
        return p


def enumerate_dvms(dim: int, Q: int, e_max: int, max_groups: int = 0,
                   scattering: bool = False) -> list:
    """All minimal DVMs of quadrature order Q with stencil energy <= e_max
    (lbm_dvm_enumerate), sorted by V, E and c: dicts with V, E, c, the
    generators and the group weights. scattering keeps stencils without a
    velocity that has a zero component."""
    flags = 1 if scattering else 0
    n = ctypes.c_int()
    rc = lib().lbm_dvm_enumerate(dim, Q, e_max, max_groups, flags, None, 0, ctypes.byref(n))
    if rc not in (LBM_OK, -3):
        check(rc, "lbm_dvm_enumerate")
    buf = (DvmModelC * max(1, n.value))()
    check(lib().lbm_dvm_enumerate(dim, Q, e_max, max_groups, flags, buf, n.value, ctypes.byref(n)),
          "lbm_dvm_enumerate")
    out = []
    for m in buf[: n.value]:
        gens = [tuple(m.gen[g * dim + k] for k in range(dim)) for g in range(m.n_groups)]
        out.append(dict(V=m.V, E=m.E, c=m.c, gens=gens, weights=list(m.w_group[: m.n_groups])))
    return out


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

    def __init__(self, dvm: Dvm, prob: Problem, device: str = "cuda", stream=None,
                 static_scratch: bool = False):
        """static_scratch: the library's static device scratch
        (lbm_solver_create_static) instead of a torch-allocated one; at most
        one such solver per device may be in use at a time."""
        import torch

        self.torch = torch
        self.dvm, self.prob = dvm, prob
        self.device = torch.device(device)
        pop_b, scr_b = state_bytes(dvm, prob)
        # 256-byte aligned allocations from torch's allocator: the population
        # buffer (one copy stepped in place, or two ping-pong) and the scratch
        self.pop = torch.empty(pop_b, dtype=torch.uint8, device=self.device)
        self.scratch = (None if static_scratch
                        else torch.empty(scr_b, dtype=torch.uint8, device=self.device))
        for t in (self.pop, self.scratch):
            if t is not None and t.data_ptr() % 256:
                raise RuntimeError("device allocation is not 256-byte aligned")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.params = params(dvm, prob)
        self.nodes = prob.nx * prob.ny * (prob.nz if prob.dim == 3 else 1)
        self.shape = ((prob.nz, prob.ny, prob.nx) if prob.dim == 3 else (prob.ny, prob.nx))
        pc = prob.to_c()
        h = _P()
        if static_scratch:
            check(lib().lbm_solver_create_static(dvm._h, ctypes.byref(pc), _ptr(self.pop),
                                                 ctypes.c_void_p(self.stream.cuda_stream),
                                                 ctypes.byref(h)),
                  "lbm_solver_create_static")
        else:
            check(lib().lbm_solver_create(dvm._h, ctypes.byref(pc), _ptr(self.pop), None,
                                          _ptr(self.scratch), scr_b,
                                          ctypes.c_void_p(self.stream.cuda_stream),
                                          ctypes.byref(h)),
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

    def set_resident_steps(self, max_steps: int):
        """Most steps per one-workgroup resident launch (small 2D problems;
        0: off)."""
        check(lib().lbm_solver_set_resident_steps(self._h, int(max_steps)),
              "lbm_solver_set_resident_steps")
        return self

    def set_pair_steps(self, on, band_rows: int = 0):
        """Two time steps per launch (2D ping-pong problems; bitwise the same
        results): on = False/0 off; True/1 all waves alternate the two steps;
        2 producer and consumer waves; 3 two producer groups on alternate
        chunks and consumer waves; band_rows 0 lets the library choose."""
        check(lib().lbm_solver_set_pair_steps(self._h, int(on), int(band_rows)),
              "lbm_solver_set_pair_steps")
        return self

    def set_graph_steps(self, max_steps: int):
        """Longest step sequence replayed from one captured HIP graph (0: one
        launch per step)."""
        check(lib().lbm_solver_set_graph_steps(self._h, int(max_steps)),
              "lbm_solver_set_graph_steps")
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

    def time_launches(self, n: int, steps_per_launch: int = 1, system_scope: bool = False):
        """Event-to-event durations (ms) of n runs of steps_per_launch steps
        each (lbm_time_launches; a measurement aid)."""
        import numpy as np
        out = np.zeros(int(n), dtype=np.float32)
        check(lib().lbm_time_launches(self._h, _P(self.stream.cuda_stream), int(n),
                                      int(steps_per_launch), int(bool(system_scope)),
                                      out.ctypes.data_as(_P)), "lbm_time_launches")
        return out

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


STATUS_NAMES = {0: "converged", -6: "not_converged", -5: "failed"}


class Batch:
    """Many independent channels (nx = 1) stepped together, each to a
    steady-state tolerance; populations resident in LDS while stepping and in
    the caller's HBM pool (a torch tensor) in between."""

    def __init__(self, max_slots: int, storage: str = "f32", pool_bytes: int = 256 << 20,
                 device: str = "cuda", stream=None):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=self.device)
        if self.pool.data_ptr() % 256:
            raise RuntimeError("pool is not 256-byte aligned")
        # graph capture needs a stream other than the legacy default stream
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.storage = storage
        self.max_slots = max_slots
        h = _P()
        check(lib().lbm_batch_create(int(max_slots), STORAGE[storage], _ptr(self.pool), int(pool_bytes),
                                     ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
              "lbm_batch_create")
        self._h = h
        self._dvms = []
        self._buf = (ResultC * max(64, max_slots * 4))()

    def submit(self, dvm: Dvm, ny: int, kn: float, ma: float = 1e-3, N: int | None = None,
               tol: float = 1e-8, check_every: int = 100, max_steps: int = 10**7,
               req_id: int = 0, rho0: float = 1.0):
        prob = Problem(dim=2, nx=1, ny=int(ny), kn=float(kn), ma=float(ma),
                       hermite_order=N if N is not None else getattr(dvm, "default_N", 3),
                       storage=self.storage, rho0=rho0)
        pc = prob.to_c()
        self._dvms.append(dvm)
        check(lib().lbm_batch_submit(self._h, dvm._h, ctypes.byref(pc), float(tol), int(check_every),
                                     int(max_steps), ctypes.c_uint64(int(req_id))), "lbm_batch_submit")

    def _results(self, n):
        out = []
        for k in range(n):
            r = self._buf[k]
            out.append(dict(req_id=int(r.req_id), status=STATUS_NAMES.get(r.status, r.status),
                            ny=r.ny, steps=int(r.steps), mdot=r.mdot, kn=r.kn))
        return out

    def _call(self, fn, name):
        res = []
        while True:
            n = ctypes.c_int()
            check(fn(self._h, self._buf, len(self._buf), ctypes.byref(n)), name)
            res += self._results(n.value)
            if n.value < len(self._buf):
                return res

    def poll(self):
        return self._call(lib().lbm_batch_poll, "lbm_batch_poll")

    def drain(self):
        return self._call(lib().lbm_batch_drain, "lbm_batch_drain")

    def run_persistent(self):
        return self._call(lib().lbm_batch_run_persistent, "lbm_batch_run_persistent")

    def tune(self, threads: int, quantum: int = 1000, slots_per_cu: int = 0, order=None):
        order = {None: 0, 0: 0, "longest_first": 1, "submit": 2}[order]
        check(lib().lbm_batch_tune(self._h, int(threads), int(quantum), int(slots_per_cu), order),
              "lbm_batch_tune")
        return self

    def autotune(self, trial_steps: int = 300) -> dict:
        """Workgroup size, resident workgroups per CU and work-queue order of
        the persistent launch, chosen by timing trials (lbm_batch_autotune)."""
        t = BatchTuningC()
        check(lib().lbm_batch_autotune(self._h, int(trial_steps), ctypes.byref(t)),
              "lbm_batch_autotune")
        return dict(threads=t.threads, slots_per_cu=t.slots_per_cu,
                    order=BATCH_ORDERS[t.order], trials=t.trials, trial_ms=round(t.trial_ms, 4))

    def stats(self):
        st = BatchStatsC()
        check(lib().lbm_batch_stats(self._h, ctypes.byref(st)), "lbm_batch_stats")
        return {f: getattr(st, f) for f, _ in BatchStatsC._fields_}

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            lib().lbm_batch_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
