"""Seeded synthetic workloads shared by tests, the smoke check and the benchmark.

Holds sizes, seeds and random draws only: none of the method's arithmetic.
The paper has no public benchmark or dataset; these inputs have the shapes and
value distributions of its plane-Poiseuille set-up (Section VI) at the sizes of
the benchmark configurations.
"""
from __future__ import annotations

import numpy as np

# Plain FP64 Poiseuille channel on D2V17: Nx=1 x Ny=40, Kn=0.1, Ma=1e-3, N=3.
CHANNEL_D2V17 = dict(dvm="D2V17", N=3, nx=1, ny=40, kn=0.1, ma=1e-3, steps=20000, storage="f64")

# Throughput channel on D2V37: 2048 x 512 periodic-x, Kn=0.05, N=4, FP32 SoA,
# rho = 1 + 1e-3 N(0,1) per node, u = 0, 1000 steps.
THROUGHPUT_D2V37 = dict(dvm="D2V37", N=4, nx=2048, ny=512, kn=0.05, ma=1e-3, steps=1000,
                        storage="f32", seed=1510, amp=1e-3)

# Batched Kn sweep: 64 D2V37 channels, Nx=1, Ny ~ U[16, 512], Kn log-uniform [0.01, 1].
SWEEP = dict(dvm="D2V37", N=4, channels=64, ny_lo=16, ny_hi=512, kn_lo=0.01, kn_hi=1.0,
             ma=1e-3, tol=1e-8, check_every=100, seed=8886)

# Serving trace: Poisson arrivals at 200/s, Ny ~ U[16, 1024], Kn log-uniform,
# DVM in {D2V17, D2V37}; 1000 requests.
SERVE = dict(rate=200.0, requests=1000, ny_lo=16, ny_hi=1024, kn_lo=0.01, kn_hi=1.0,
             dvms=("D2V17", "D2V37"), ma=1e-3, tol=1e-8, check_every=100, seed=2426)

# 3D square duct on D3V39: 128 x 256 x 256, walls on y and z, Kn=0.1, N=3.
DUCT_D3V39 = dict(dvm="D3V39", N=3, nx=128, ny=256, nz=256, kn=0.1, ma=1e-3, steps=500)
# scattering stencils at the channel / duct sizes above (FP32 populations)
SCATTER_D2V32 = dict(dvm="D2V32", N=4, nx=2048, ny=512, kn=0.05, ma=1e-3, steps=200)
SCATTER_D3V96 = dict(dvm="D3V96", N=3, nx=128, ny=256, nz=256, kn=0.1, ma=1e-3, steps=50)


def density_field(ny: int, nx: int, seed: int = 1510, amp: float = 1e-3) -> np.ndarray:
    """rho = 1 + amp * N(0,1) per node, y-major / x-fastest order."""
    rng = np.random.default_rng(seed)
    return 1.0 + amp * rng.standard_normal(ny * nx)


def sweep_channels(n: int = 64, seed: int = 8886, ny_lo: int = 16, ny_hi: int = 512,
                   kn_lo: float = 0.01, kn_hi: float = 1.0):
    """Per channel, drawn in this order: Ny = integers(ny_lo, ny_hi + 1),
    Kn = 10 ** uniform(log10 kn_lo, log10 kn_hi)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        ny = int(rng.integers(ny_lo, ny_hi + 1))
        kn = float(10 ** rng.uniform(np.log10(kn_lo), np.log10(kn_hi)))
        out.append(dict(ny=ny, kn=kn))
    return out


def serve_trace(n: int = 1000, seed: int = 2426, rate: float = 200.0, ny_lo: int = 16,
                ny_hi: int = 1024, kn_lo: float = 0.01, kn_hi: float = 1.0,
                dvms=("D2V17", "D2V37")):
    """Requests with Poisson arrival times (s), Ny, Kn and DVM name."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n):
        t += float(rng.exponential(1.0 / rate))
        ny = int(rng.integers(ny_lo, ny_hi + 1))
        kn = float(10 ** rng.uniform(np.log10(kn_lo), np.log10(kn_hi)))
        name = str(rng.choice(list(dvms)))
        out.append(dict(id=k, t=t, ny=ny, kn=kn, dvm=name))
    return out


def random_state(nodes: int, dim: int, seed: int, amp: float):
    """Density and velocity perturbations for small parity cases."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + amp * rng.standard_normal(nodes)
    u = np.zeros((nodes, 3))
    u[:, :dim] = amp * rng.standard_normal((nodes, dim))
    return rho, u
