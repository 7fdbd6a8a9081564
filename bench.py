#!/usr/bin/env python3
"""Benchmark of the fused stream + wall + collide step on one MI355X.

Workload: the D2V37 FP32 throughput channel, 2048 x 512 nodes (periodic x,
diffuse Maxwell walls at y), Kn = 0.05, Hermite order 4, seeded density
1 + 1e-3 N(0,1), u = 0. One benchmark step = one lattice update of the whole
grid. Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

import lbm_workloads as wl  # noqa: E402

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = ROOT / "profiles" / "traffic_step_d2v37_f32_2048x512.json"
KERNEL_SOURCES = ["paper_1510_08886_amd/csrc/lbm_kernels.hip",
                  "paper_1510_08886_amd/csrc/lbm_device.h",
                  "paper_1510_08886_amd/csrc/lbm_internal.h",
                  "paper_1510_08886_amd/csrc/lbm_sets.h"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for s in KERNEL_SOURCES:
        h.update((ROOT / s).read_bytes())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter runs, only if
    they were taken on the current kernel source."""
    if not TRAFFIC_FILE.exists():
        return None
    try:
        rec = json.loads(TRAFFIC_FILE.read_text())
    except ValueError:
        return None
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(budget_s: float = 20.0):
    """The FP64 oracle on the same grid and seeded input, all host threads."""
    import numpy as np

    from oracle import dvm as odvm
    from oracle import stepper

    c = wl.THROUGHPUT_D2V37
    threads = min(os.cpu_count() or 1, 64)
    o = stepper.OracleSolver(odvm.named_dvm(c["dvm"]), nx=c["nx"], ny=c["ny"], kn=c["kn"],
                             ma=c["ma"], N=c["N"])
    o.init(rho=wl.density_field(c["ny"], c["nx"], seed=c["seed"], amp=c["amp"]))
    t0 = time.perf_counter()
    o.run(1, nthreads=threads)
    one = time.perf_counter() - t0
    steps = max(1, min(50, int(budget_s / max(one, 1e-3)) - 1))
    t0 = time.perf_counter()
    o.run(steps, nthreads=threads)
    el = time.perf_counter() - t0
    nodes = c["nx"] * c["ny"]
    return {"value": nodes * steps / el / 1e6, "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"{steps} steps of the full 2048x512 D2V37 grid in FP64 "
                      f"(after 1 warm-up step), {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=wl.THROUGHPUT_D2V37["steps"])
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of the same byte count (for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; "
                                   f"--gpus {args.gpus} is not supported"}))
        sys.exit(2)

    import torch

    from paper_1510_08886_amd import lbm

    c = wl.THROUGHPUT_D2V37
    if args.copy_calibration:
        # one plain copy kernel moving the bytes of one lattice update
        n = 37 * c["nx"] * c["ny"]
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": 4 * n, "copy_calibration_bytes_written": 4 * n,
                          "launches": 3}))
        return
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    d = lbm.Dvm.named(c["dvm"])
    prob = lbm.Problem(dim=2, nx=c["nx"], ny=c["ny"], kn=c["kn"], ma=c["ma"], hermite_order=c["N"],
                       storage=c["storage"])
    s = lbm.Solver(d, prob, device="cuda:0")
    rho = torch.from_numpy(wl.density_field(c["ny"], c["nx"], seed=c["seed"], amp=c["amp"]))
    s.init(rho)
    s.run(args.warmup)
    stream = s.stream
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t0 = time.perf_counter()
    s.run(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    nodes = c["nx"] * c["ny"]
    mlups = nodes * args.steps / (ms * 1e-3) / 1e6
    bytes_per_launch = 2 * d.V * 4 * nodes         # each population read once, written once
    achieved = bytes_per_launch / (ms * 1e-3 / args.steps) / 1e9
    obs = s.observe()
    out = {
        "metric": "MLUPS (fused stream+collide, D2V37 FP32 channel) & % HBM peak",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "D2V37 FP32 Poiseuille channel 2048x512, Kn=0.05, N=4, "
                               "seeded rho=1+1e-3*N(0,1)",
                   "nx": c["nx"], "ny": c["ny"], "V": d.V, "storage": "f32",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic()},
        "wall_s": round(wall, 3),
        "mdot_after": obs["mdot"],
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
