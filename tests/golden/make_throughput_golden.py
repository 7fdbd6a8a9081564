"""Writes throughput_d2v37.txt: the FP64 oracle's run of the 2048 x 512 D2V37
throughput channel (Hermite order 4, Kn = 0.05, Ma = 1e-3 body force, diffuse
Maxwell walls at both y walls, periodic x), started at equilibrium with the
seeded density rho = 1 + 1e-3 N(0,1) per node and u = 0, for 1000 steps.

Stored: the mass flow (Eq. pf.1) and total mass every 100 steps; after the last
step the row average of u_x at every row, and rho, u_x, u_y of the streamed
state (Eq. nm.10) on four sampled columns. The density field comes from the
seeded recipe in lbm_workloads; only the oracle is called.

    python -m tests.golden.make_throughput_golden [--threads N]
"""
from __future__ import annotations

import argparse
import time
from pathlib import Path

import numpy as np

import lbm_workloads as wl
from oracle import dvm as odvm
from oracle import stepper

OUT = Path(__file__).resolve().parent / "throughput_d2v37.txt"
EVERY = 100
COLUMNS = (0, 511, 1024, 2047)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    c = wl.THROUGHPUT_D2V37
    rho = wl.density_field(c["ny"], c["nx"], seed=c["seed"], amp=c["amp"])
    o = stepper.OracleSolver(odvm.named_dvm(c["dvm"]), nx=c["nx"], ny=c["ny"], kn=c["kn"],
                             ma=c["ma"], N=c["N"]).init(rho=rho)
    lines = ["# FP64 oracle, D2V37 N = 4 channel 2048 x 512, Kn = 0.05, Ma = 1e-3, from",
             "# equilibrium at rho = 1 + 1e-3 N(0,1) (default_rng(1510), y-major), u = 0;",
             "# written by tests/golden/make_throughput_golden.py, which calls only the oracle.",
             f"steps {c['steps']}", f"columns {' '.join(str(i) for i in COLUMNS)}"]
    t0 = time.time()
    done = 0
    ob = None
    while done < c["steps"]:
        o.run(EVERY, nthreads=a.threads)
        done += EVERY
        ob = o.observe()
        lines.append(f"mdot {done} {ob['mdot']!r} {ob['mass']!r}")
        print(f"step {done} mdot {ob['mdot']:.17e} ({time.time() - t0:.0f} s)", flush=True)
    ux_row = ob["u"][..., 0].mean(axis=1)
    lines += [f"uxrow {j} {float(v)!r}" for j, v in enumerate(ux_row)]
    for i in COLUMNS:
        for j in range(c["ny"]):
            lines.append(f"col {i} {j} {float(ob['rho'][j, i])!r} {float(ob['u'][j, i, 0])!r} "
                         f"{float(ob['u'][j, i, 1])!r}")
    OUT.write_text("\n".join(lines) + "\n")
    print(f"wrote {OUT} ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
