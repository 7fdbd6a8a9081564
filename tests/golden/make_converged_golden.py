"""Writes the FP64 oracle's converged mass flows of the batched Kn sweep (all
64 channels) and of a seeded sample of the serving trace.

Each solve is the plane Poiseuille channel of Section VI (nx = 1, diffuse
Maxwell walls, Ma = 1e-3 body force, from rest), stepped by the oracle until
the relative change of the mass flow (Eq. pf.1) between two evaluations 100
steps apart is below 1e-8 (the convergence test the GPU engine applies, with
the same check points), then for WINDOW_AFTER more steps. The file records the
oracle's stop step and the mass flow at every check point up to WINDOW_AFTER
steps after the stop: the transient oscillates, so a run in another precision
may meet the tolerance at a check thousands of steps earlier or later than
the oracle does, and it is compared at its own step.

Serving sample: requests of the seeded trace (lbm_workloads.serve_trace) in
four Ny quarters of [16, 1024] and both DVMs, SAMPLE_PER_CELL per (DVM,
quarter), drawn by default_rng(SAMPLE_SEED) among the requests whose oracle
cost estimate 2.1 ny^2 / Kn lattice updates (a diffusion time to converge) is
below COST_CAP for its DVM. Only the oracle and the seeded recipes are called.

    python -m tests.golden.make_converged_golden [--procs N] [--only sweep|serve]
"""
from __future__ import annotations

import argparse
import time
from multiprocessing import Pool
from pathlib import Path

import numpy as np

import lbm_workloads as wl

HERE = Path(__file__).resolve().parent
OUT_SWEEP = HERE / "sweep_d2v37_converged.txt"
OUT_SERVE = HERE / "serve_sample_converged.txt"
CHECK = 100
TOL = 1e-8
WINDOW_AFTER = 3000
MAX_STEPS = 2_000_000
SAMPLE_SEED = 5901
SAMPLE_PER_CELL = 5
COST_CAP = {"D2V37": 2.5e7, "D2V17": 1.2e8}
N_OF = {"D2V17": 3, "D2V37": 4}


def solve(job):
    """(key, dvm, ny, kn) -> key, stop step, [(step, mdot)] at every check."""
    from oracle import dvm as odvm
    from oracle import stepper

    key, name, ny, kn = job
    t0 = time.time()
    o = stepper.OracleSolver(odvm.named_dvm(name), nx=1, ny=ny, kn=kn, ma=1e-3,
                             N=N_OF[name]).init()
    hist = []
    prev = None
    stop = None
    steps = 0
    while steps < MAX_STEPS:
        o.run(CHECK, nthreads=1)
        steps += CHECK
        m = o.observe()["mdot"]
        hist.append((steps, m))
        if stop is None and prev is not None and abs(m - prev) < TOL * abs(m):
            stop = steps
        prev = m
        if stop is not None and steps >= stop + WINDOW_AFTER:
            break
    return key, name, ny, kn, stop, hist, time.time() - t0


def sweep_jobs():
    c = wl.SWEEP
    chans = wl.sweep_channels(c["channels"], seed=c["seed"], ny_lo=c["ny_lo"], ny_hi=c["ny_hi"],
                              kn_lo=c["kn_lo"], kn_hi=c["kn_hi"])
    return [(k, c["dvm"], ch["ny"], ch["kn"]) for k, ch in enumerate(chans)]


def serve_sample():
    c = wl.SERVE
    trace = wl.serve_trace(c["requests"], seed=c["seed"], rate=c["rate"], ny_lo=c["ny_lo"],
                           ny_hi=c["ny_hi"])
    rng = np.random.default_rng(SAMPLE_SEED)
    edges = np.linspace(c["ny_lo"], c["ny_hi"] + 1, 5)
    picked = []
    for name in c["dvms"]:
        for q in range(4):
            cell = [r for r in trace if r["dvm"] == name and edges[q] <= r["ny"] < edges[q + 1]
                    and 2.1 * r["ny"] ** 2 / r["kn"] <= COST_CAP[name]]
            take = rng.choice(len(cell), size=min(SAMPLE_PER_CELL, len(cell)), replace=False)
            picked += [cell[int(t)] for t in sorted(take)]
    return [(r["id"], r["dvm"], r["ny"], r["kn"]) for r in picked]


def write(path, title, rows):
    lines = [f"# FP64 oracle, {title}; nx = 1, Ma = 1e-3, from rest; converged when the",
             f"# relative change of mdot between checks {CHECK} steps apart is below {TOL:g};",
             "# written by tests/golden/make_converged_golden.py, which calls only the oracle.",
             "# solve <key> <dvm> <ny> <kn> <stop step>, then mdot <step> <value> lines"]
    for key, name, ny, kn, stop, window, _ in sorted(rows):
        lines.append(f"solve {key} {name} {ny} {kn!r} {stop}")
        lines += [f"mdot {s} {m!r}" for s, m in window]
    path.write_text("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=8)
    ap.add_argument("--only", choices=["sweep", "serve"], default=None)
    a = ap.parse_args()
    todo = []
    if a.only in (None, "sweep"):
        todo.append((OUT_SWEEP, "64-channel D2V37 N = 4 Kn sweep (default_rng(8886))", sweep_jobs()))
    if a.only in (None, "serve"):
        todo.append((OUT_SERVE, "sample of the serving trace (default_rng(2426)), "
                                f"{SAMPLE_PER_CELL} per DVM and Ny quarter", serve_sample()))
    for path, title, jobs in todo:
        # longest first, so the pool drains evenly
        jobs = sorted(jobs, key=lambda j: -(j[2] ** 2 / j[3]) * (5 if j[1] == "D2V37" else 1))
        rows = []
        with Pool(a.procs) as pool:
            for r in pool.imap_unordered(solve, jobs):
                rows.append(r)
                print(f"{path.name}: {len(rows)}/{len(jobs)} key {r[0]} {r[1]} ny {r[2]} "
                      f"kn {r[3]:.4f} stop {r[4]} ({r[6]:.0f} s)", flush=True)
        write(path, title, rows)


if __name__ == "__main__":
    main()
