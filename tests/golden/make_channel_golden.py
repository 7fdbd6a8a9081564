"""Writes channel_d2v17.txt: the FP64 oracle's plane Poiseuille channel on
D2V17 (Hermite order 3, nx = 1, ny = 40, Kn = 0.1, Ma = 1e-3 body force,
diffuse Maxwell walls, from rest) after 20000 steps: the mass flow, the total
mass and the streamwise velocity at every node. Only the oracle is called.

    python -m tests.golden.make_channel_golden
"""
from __future__ import annotations

from pathlib import Path

import lbm_workloads as wl
from oracle import dvm as odvm
from oracle import stepper

OUT = Path(__file__).resolve().parent / "channel_d2v17.txt"


def main():
    c = wl.CHANNEL_D2V17
    o = stepper.OracleSolver(odvm.named_dvm(c["dvm"]), nx=c["nx"], ny=c["ny"], kn=c["kn"],
                             ma=c["ma"], N=c["N"]).init()
    o.run(c["steps"])
    ob = o.observe()
    ux = ob["u"][:, 0, 0]
    lines = ["# FP64 oracle, D2V17 N = 3 channel, nx = 1, ny = 40, Kn = 0.1, Ma = 1e-3, from rest;",
             "# written by tests/golden/make_channel_golden.py, which calls only the oracle.",
             f"steps {c['steps']}", f"mdot {ob['mdot']!r}", f"mass {ob['mass']!r}"]
    lines += [f"ux {j} {float(v)!r}" for j, v in enumerate(ux)]
    OUT.write_text("\n".join(lines) + "\n")
    print("\n".join(lines[:6]))


if __name__ == "__main__":
    main()
