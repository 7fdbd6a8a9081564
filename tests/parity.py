"""Helpers for GPU-vs-oracle parity: identical seeded inputs on both sides,
populations compared velocity by velocity (the two sides order velocities
differently, so they are matched by their integer vectors)."""
import numpy as np

from oracle import dvm as odvm
from oracle import stepper


def oracle_perm(lib_dvm, o_dvm):
    index = {tuple(int(x) for x in e): k for k, e in enumerate(o_dvm.velocities)}
    return np.array([index[tuple(int(x) for x in e)] for e in lib_dvm.velocities])


# velocity sets with compiled kernels that are not among the named ones:
# (dim, generators, quadrature order); both sides solve for c and the weights
EXTRA_SETS = {"D3V15": (3, [(0, 0, 0), (2, 0, 0), (1, 1, 1)], 5)}


# scattering stencils with compiled kernels, built on both sides from the
# paper's printed tables (c and weights)
TABLE_SETS = ("D2V32", "D3V96", "D2V16", "D2V33")


def dvm_pair(name):
    from paper_1510_08886_amd import lbm

    if name in TABLE_SETS:
        from tests.golden.tables import load_dvm_tables
        m = {t["label"]: t for t in load_dvm_tables()}[name]
        return (lbm.Dvm(m["D"], m["gens"], m["weights"], m["c"], m["Q"]),
                odvm.make_dvm(m["D"], m["gens"], m["weights"], m["c"], m["Q"]))
    if name in EXTRA_SETS:
        dim, gens, Q = EXTRA_SETS[name]
        return lbm.Dvm.solve(dim, gens, Q), odvm.solve_dvm(dim, gens, Q)
    return lbm.Dvm.named(name), odvm.named_dvm(name)


def make_pair(name, N, nx, ny, nz=1, kn=0.1, ma=1e-3, storage="f64", rho=None, u=None,
              walls_z=False, layout="auto", alpha=1.0):
    import torch
    from paper_1510_08886_amd import lbm

    d, od = dvm_pair(name)
    prob = lbm.Problem(dim=d.dim, nx=nx, ny=ny, nz=nz, kn=kn, ma=ma, hermite_order=N,
                       storage=storage, layout=layout, accommodation=alpha)
    g = lbm.Solver(d, prob)
    o = stepper.OracleSolver(od, nx=nx, ny=ny, nz=nz, kn=kn, ma=ma, N=N,
                             walls_z=walls_z or d.dim == 3, alpha=alpha)
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
