"""Writes sweep_d2v37_mdot.txt: the FP64 oracle's mass flow of the six
channels with the fewest rows of the 64-channel D2V37 Kn sweep (Hermite order
4, Ma = 1e-3, nx = 1, from rest), after a fixed number of steps. The channels
come from the seeded sweep recipe; only the oracle is called.

    python -m tests.golden.make_sweep_golden
"""
from __future__ import annotations

from pathlib import Path

import lbm_workloads as wl
from oracle import dvm as odvm
from oracle import stepper

OUT = Path(__file__).resolve().parent / "sweep_d2v37_mdot.txt"
STEPS = 4000
COUNT = 6


def channels():
    """(index in the sweep, ny, kn) of the COUNT channels with the fewest rows."""
    c = wl.SWEEP
    chans = wl.sweep_channels(c["channels"], seed=c["seed"], ny_lo=c["ny_lo"], ny_hi=c["ny_hi"],
                              kn_lo=c["kn_lo"], kn_hi=c["kn_hi"])
    order = sorted(range(len(chans)), key=lambda k: (chans[k]["ny"], k))[:COUNT]
    return [(k, chans[k]["ny"], chans[k]["kn"]) for k in order]


def main():
    c = wl.SWEEP
    rows = []
    for k, ny, kn in channels():
        o = stepper.OracleSolver(odvm.named_dvm(c["dvm"]), nx=1, ny=ny, kn=kn, ma=c["ma"],
                                 N=c["N"]).init()
        o.run(STEPS)
        rows.append((k, ny, kn, STEPS, o.observe()["mdot"]))
    lines = ["# FP64 oracle mass flow of the sweep channels with the fewest rows (D2V37, N = 4,",
             "# Ma = 1e-3, nx = 1, from rest) after a fixed step count; written by",
             "# tests/golden/make_sweep_golden.py, which calls only the oracle.",
             "# index ny kn steps mdot"]
    lines += [f"{k} {ny} {kn!r} {s} {m!r}" for k, ny, kn, s, m in rows]
    OUT.write_text("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
