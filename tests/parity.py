"""Helpers for GPU-vs-oracle parity: identical seeded inputs on both sides,
populations compared velocity by velocity (the two sides order velocities
differently, so they are matched by their integer vectors)."""
import numpy as np

from oracle import dvm as odvm
from oracle import stepper


def oracle_perm(lib_dvm, o_dvm):
    index = {tuple(int(x) for x in e): k for k, e in enumerate(o_dvm.velocities)}
    return np.array([index[tuple(int(x) for x in e)] for e in lib_dvm.velocities])


def make_pair(name, N, nx, ny, nz=1, kn=0.1, ma=1e-3, storage="f64", rho=None, u=None,
              walls_z=False):
    import torch
    from paper_1510_08886_amd import lbm

    spec = lbm.NAMED_DVMS[name]
    d = lbm.Dvm.named(name)
    prob = lbm.Problem(dim=spec["dim"], nx=nx, ny=ny, nz=nz, kn=kn, ma=ma, hermite_order=N,
                       storage=storage)
    g = lbm.Solver(d, prob)
    o = stepper.OracleSolver(odvm.named_dvm(name), nx=nx, ny=ny, nz=nz, kn=kn, ma=ma, N=N,
                             walls_z=walls_z or spec["dim"] == 3)
    if rho is None:
        g.init()
        o.init()
    else:
        g.init(torch.from_numpy(np.asarray(rho)), None if u is None else torch.from_numpy(np.asarray(u)))
        o.init(rho=rho, u=u)
    return d, g, o


def populations_both(d, g, o):
    pg = g.export().cpu().numpy()
    po = o.populations()[oracle_perm(d, o.dvm)]
    return pg, po
