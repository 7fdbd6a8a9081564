"""Writes duct_d3v39_mdot.txt: the FP64 oracle's mass flow of the square-duct
flow on D3V39 (Hermite order 3, Kn = 0.1, Ma = 1e-3 body force, diffuse Maxwell
walls on the four y and z faces), started from rest, 256 x 256 cross-section.

Body force along the periodic x axis and a uniform initial state keep every
x column identical, so the oracle runs one column (nx = 1); the result is the
mass flow of the duct at any nx. Only the oracle is called.

    python -m tests.golden.make_duct_golden [--threads N]
"""
from __future__ import annotations

import argparse
import time
from pathlib import Path

from oracle import dvm as odvm
from oracle import stepper

OUT = Path(__file__).resolve().parent / "duct_d3v39_mdot.txt"
NY = NZ = 256
KN, MA, N = 0.1, 1e-3, 3
STEPS, EVERY = 500, 50


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    o = stepper.OracleSolver(odvm.named_dvm("D3V39"), nx=1, ny=NY, nz=NZ, kn=KN, ma=MA, N=N,
                             walls_z=True).init()
    rows = []
    t0 = time.time()
    done = 0
    while done < STEPS:
        o.run(EVERY, nthreads=a.threads)
        done += EVERY
        ob = o.observe()
        rows.append((done, ob["mdot"], ob["mass"]))
        print(f"step {done} mdot {ob['mdot']:.17e} ({time.time() - t0:.0f} s)", flush=True)
    with open(OUT, "w") as f:
        f.write("# FP64 oracle, D3V39 N=3 square duct nx=1 ny=256 nz=256, Kn=0.1, Ma=1e-3,\n")
        f.write("# from rest; written by tests/golden/make_duct_golden.py\n")
        f.write("# step mdot mass\n")
        for s, m, ms in rows:
            f.write(f"{s} {m:.17e} {ms:.17e}\n")


if __name__ == "__main__":
    main()
