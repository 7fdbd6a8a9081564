#!/usr/bin/env python3
"""Benchmark of the fused stream + wall + collide step on one MI355X.

Headline: the D2V37 FP32 throughput channel, 2048 x 512 nodes (periodic x,
diffuse Maxwell walls at y), Kn = 0.05, Hermite order 4, seeded density
1 + 1e-3 N(0,1), u = 0, stepped as the library does by default (two ping-pong
copies, two lattice updates per launch). One benchmark step = one lattice
update of the whole grid: MLUPS and the HBM roofline fraction against the
algorithmic 2 V s bytes per update, with the bytes the kernel moves beside it;
the one-step in-place kernels on the same channel are reported too. Also reported on the same line: the
batched 64-channel Kn sweep (solves/s vs one solve at a time with plain
kernels), the served 1000-request trace (p50/p99 latency, solves/s) and the
3D D3V39 duct with FP32 and FP16-deviation populations. Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

import lbm_workloads as wl  # noqa: E402

HBM_PEAK_GBS = 8000.0
# the 256 MB last-level cache (Infinity Cache) of one MI355X
LLC_BYTES = 256 * 2**20
# the headline's kernel (two steps per launch), the same channel's one-step
# in-place kernels, and the two-step kernel on the above-cache channel
HEAD_TRAFFIC_FILE = ROOT / "profiles" / "traffic_pair_d2v37_f32_2048x512.json"
TRAFFIC_FILE = ROOT / "profiles" / "traffic_step_d2v37_f32_2048x512.json"
PAIR_TRAFFIC_FILE = ROOT / "profiles" / "traffic_pair_d2v37_f32_4096x2048.json"
# what the headline kernels' traffic depends on: their sources, the device
# compiler flags and the host's choice between in-place and ping-pong stepping
KERNEL_SOURCES = ["paper_1510_08886_amd/csrc/lbm_kernels.hip",
                  "paper_1510_08886_amd/csrc/lbm_device.h",
                  "paper_1510_08886_amd/csrc/lbm_node2d.h",
                  "paper_1510_08886_amd/csrc/lbm_internal.h",
                  "paper_1510_08886_amd/csrc/lbm_sets.h",
                  "paper_1510_08886_amd/csrc/lbm_api.cpp"]


_TOKENS = re.compile(r'"(?:\\.|[^"\\\n])*"|//[^\n]*|/\*.*?\*/', re.S)


def _code_only(src: str) -> str:
    """C/C++ source without comments, whitespace runs collapsed."""
    src = _TOKENS.sub(lambda m: m.group(0) if m.group(0).startswith('"') else " ", src)
    return " ".join(src.split())


def kernel_hash() -> str:
    from paper_1510_08886_amd.build import HIPCC_FLAGS
    h = hashlib.sha256()
    for s in KERNEL_SOURCES:
        h.update(_code_only((ROOT / s).read_text()).encode())
    h.update(" ".join(HIPCC_FLAGS).encode())
    return h.hexdigest()[:16]


def profile_record(path=TRAFFIC_FILE):
    """The committed rocprofv3 record of a kernel (counter bytes per launch,
    trace time per launch), only if it was taken on the current kernel
    source."""
    if not path.exists():
        return None
    try:
        rec = json.loads(path.read_text())
    except ValueError:
        return None
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec


def measured_traffic(path=TRAFFIC_FILE):
    """HBM bytes per launch from the committed counter runs (or None)."""
    rec = profile_record(path)
    return None if rec is None else rec.get("bytes_per_launch")


def _cpu_model() -> str:
    try:
        for line in Path("/proc/cpuinfo").read_text().splitlines():
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(budget_s: float = 15.0):
    """The FP64 oracle on the same grid and seeded input: one step on one
    thread, then as many steps as fit the budget on all the host threads this
    process may use."""
    from oracle import dvm as odvm
    from oracle import stepper

    c = wl.THROUGHPUT_D2V37
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = max(1, min(avail or 1, 64))
    o = stepper.OracleSolver(odvm.named_dvm(c["dvm"]), nx=c["nx"], ny=c["ny"], kn=c["kn"],
                             ma=c["ma"], N=c["N"])
    o.init(rho=wl.density_field(c["ny"], c["nx"], seed=c["seed"], amp=c["amp"]))
    nodes = c["nx"] * c["ny"]
    t0 = time.perf_counter()
    o.run(1, nthreads=1)
    one_thread_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    o.run(1, nthreads=threads)
    one = time.perf_counter() - t0
    steps = max(1, min(50, int(budget_s / max(one, 1e-3))))
    t0 = time.perf_counter()
    o.run(steps, nthreads=threads)
    el = time.perf_counter() - t0
    return {"value": nodes * steps / el / 1e6, "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"{steps} steps of the full 2048x512 D2V37 grid in FP64 on {threads} "
                      f"threads (after 1 warm-up step), {el:.1f} s; 1 step on 1 thread, "
                      f"{one_thread_s:.1f} s",
            "one_thread_mlups": round(nodes / one_thread_s / 1e6, 4),
            "nproc": os.cpu_count(), "cpu_model": _cpu_model()}


def throughput_parity(d, prob):
    """The headline workload run untimed for exactly its 1000 steps from the
    seeded density, against the stored FP64 oracle run of the same channel
    (tests/golden/throughput_d2v37.txt, written by a script that calls only the
    oracle): relative error of the mass flow (Eq. pf.1), of the row-averaged
    u_x, of rho on the stored columns (elementwise), and of u_x, u_y there
    relative to the column's largest |u_x|, the scale of the flow (FP32
    deviation storage errs on the velocity by an amount set by the flow, so
    u_y, a thousand times smaller than u_x here, is held to the flow's scale;
    its error relative to its own largest magnitude is reported beside)."""
    import numpy as np
    import torch

    from paper_1510_08886_amd import lbm

    c = wl.THROUGHPUT_D2V37
    g = {"uxrow": {}, "col": {}}
    for line in (ROOT / "tests" / "golden" / "throughput_d2v37.txt").read_text().splitlines():
        t = line.split()
        if not t or t[0].startswith("#"):
            continue
        if t[0] == "mdot" and int(t[1]) == c["steps"]:
            g["mdot"] = float(t[2])
        elif t[0] == "uxrow":
            g["uxrow"][int(t[1])] = float(t[2])
        elif t[0] == "col":
            g["col"][(int(t[1]), int(t[2]))] = [float(x) for x in t[3:6]]
    s = lbm.Solver(d, prob, device="cuda:0")
    s.init(torch.from_numpy(wl.density_field(c["ny"], c["nx"], seed=c["seed"], amp=c["amp"])))
    s.run(c["steps"])
    ob = s.observe()
    s.close()
    u, r = ob["u"].cpu().numpy(), ob["rho"].cpu().numpy()
    want_row = np.array([g["uxrow"][j] for j in range(c["ny"])])
    row_err = float(np.max(np.abs(u[..., 0].mean(axis=1) - want_row)) / np.max(np.abs(want_row)))
    field_err = uy_own = 0.0
    for i in sorted({i for i, _ in g["col"]}):
        ref = np.array([g["col"][(i, j)] for j in range(c["ny"])])
        field_err = max(field_err, float(np.max(np.abs(r[:, i] - ref[:, 0]) / ref[:, 0])))
        scale = np.max(np.abs(ref[:, 1]))
        for k in (1, 2):
            field_err = max(field_err, float(np.max(np.abs(u[:, i, k - 1] - ref[:, k])) / scale))
        uy_own = max(uy_own, float(np.max(np.abs(u[:, i, 1] - ref[:, 2])) / np.max(np.abs(ref[:, 2]))))
    return {"steps": c["steps"], "mdot": ob["mdot"], "oracle_mdot": g["mdot"],
            "mdot_rel_err_vs_oracle": abs(ob["mdot"] - g["mdot"]) / abs(g["mdot"]),
            "ux_row_rel_err": row_err, "sampled_fields_rel_err": field_err,
            "sampled_uy_rel_err_own_scale": uy_own}


def copy_gbs(nbytes: int, reps: int = 10) -> float:
    """Bandwidth of the library's plain streaming copy (one 16-byte vector per
    thread, non-temporal stores) of nbytes each way, alternating direction
    between two buffers so that every copy reads what the previous one wrote
    (as a step does): the practical ceiling a streaming kernel of the same
    footprint reaches on this part, next to the 8 TB/s peak."""
    import torch

    from paper_1510_08886_amd import lbm
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()
    for k in range(4):
        lbm.stream_copy(*((a, b) if k % 2 == 0 else (b, a)), st)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for k in range(reps):
        lbm.stream_copy(*((a, b) if k % 2 == 0 else (b, a)), st)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * 4 * n / (ms * 1e-3) / 1e9


def _err_stats(errs):
    import numpy as np
    e = np.array([x for x in errs if x is not None])
    return {"channels": int(len(e)), "missing": int(sum(x is None for x in errs)),
            "max": float(e.max()) if len(e) else None,
            "median": float(np.median(e)) if len(e) else None}


def _sweep_errors(res, gold):
    from tests.golden.converged import rel_err_at
    return [rel_err_at(gold[k], r["steps"], r["mdot"]) if k in gold else None
            for k, r in enumerate(res)]


def batched_block():
    """64-channel D2V37 Kn sweep to a 1e-8 tolerance. Primary: FP32 deviations
    collided in FP64 with stochastic rounding (f32sr, the storage that meets
    the FP32 mass-flux tolerance), one persistent launch (autotuned, graph
    replayed) against the same solves one at a time through the single-solve
    path at the same storage (equal accuracy). Beside it: plain FP32 (FP32
    collision, round to nearest) and FP16 deviations (stepped to the f32sr
    stop steps). Every channel's mass flow is compared with the stored FP64
    oracle value at its own stop step."""
    from paper_1510_08886_amd import serve
    from tests.golden.converged import SWEEP, load_converged
    cfg = wl.SWEEP
    chans = wl.sweep_channels(cfg["channels"], seed=cfg["seed"])
    gold = load_converged(SWEEP) if SWEEP.exists() else {}
    for k, g in gold.items():
        assert (chans[k]["ny"], chans[k]["kn"]) == (g["ny"], g["kn"]), "sweep recipe changed"
    kw = dict(tol=cfg["tol"], check_every=cfg["check_every"])
    sr = serve.batched_sweep(chans, storage="f32sr", **kw)
    steps = [r["steps"] for r in sr["results"]]
    plain = serve.plain_sweep(chans, storage="f32sr", **kw)
    same = all(a["steps"] == b["steps"] and abs(a["mdot"] - b["mdot"]) <= 1e-13 * abs(b["mdot"])
               for a, b in zip(sr["results"], plain["results"]))
    f32 = serve.batched_sweep(chans, storage="f32", **kw)
    # FP16 stochastic rounding keeps a noise floor above a 1e-8 relative
    # change per check, so FP16 runs each channel to the f32sr stop step
    f16 = serve.batched_sweep(chans, storage="f16dev", tol=1e-300, check_every=cfg["check_every"],
                              max_steps=steps)
    assert [r["steps"] for r in f16["results"]] == steps
    conv = [abs(r["mdot"] - gold[k]["mdot"][gold[k]["stop"]]) / abs(gold[k]["mdot"][gold[k]["stop"]])
            if k in gold and gold[k]["stop"] else None for k, r in enumerate(sr["results"])]
    stop_diff = [r["steps"] - gold[k]["stop"] for k, r in enumerate(sr["results"])
                 if k in gold and gold[k]["stop"]]
    n = len(chans)
    note = "every channel against the stored FP64 oracle mass flow at its own stop step"
    return {
        "workload": "64 D2V37 channels, Nx=1, Ny~U[16,512], Kn log-uniform [0.01,1], Ma=1e-3, "
                    "tol 1e-8 on mdot every 100 steps",
        "storage": "f32sr (FP32 deviations, FP64 collision, stochastic rounding)",
        "solves_per_s": round(n / sr["makespan_s"], 2),
        "makespan_s": round(sr["makespan_s"], 4),
        "plain_solves_per_s": round(n / plain["total_s"], 2),
        "plain_total_s": round(plain["total_s"], 3),
        "speedup_vs_plain": round(plain["total_s"] / sr["makespan_s"], 2),
        "converged": sum(r["status"] == "converged" for r in sr["results"]),
        "total_steps": int(sum(steps)),
        "autotune": dict(sr["tuning"], tune_s=round(sr["tune_s"], 3)),
        "graph_replays": sr["graph_replays"],
        "batched_equals_plain": bool(same),
        "mdot_rel_err_vs_oracle": dict(_err_stats(_sweep_errors(sr["results"], gold)), note=note),
        "mdot_rel_err_vs_oracle_converged": _err_stats(conv),
        "stop_step_minus_oracle_stop": {"min": min(stop_diff, default=None),
                                        "max": max(stop_diff, default=None)},
        "f32": {"storage": "FP32 deviations, FP32 collision, round to nearest",
                "makespan_s": round(f32["makespan_s"], 4),
                "solves_per_s": round(n / f32["makespan_s"], 2),
                "converged": sum(r["status"] == "converged" for r in f32["results"]),
                "mdot_rel_err_vs_oracle": dict(_err_stats(_sweep_errors(f32["results"], gold)),
                                               note=note),
                "autotune": f32["tuning"]},
        "fp16dev": {"makespan_s": round(f16["makespan_s"], 4),
                    "solves_per_s": round(n / f16["makespan_s"], 2),
                    "steps": "the f32sr stop step of each channel",
                    "mdot_rel_err_vs_oracle": dict(_err_stats(_sweep_errors(f16["results"], gold)),
                                                   note=note),
                    "autotune": f16["tuning"]},
    }


# the served engine's storage: the one that meets the FP32 mass-flux tolerance
STORAGE_SERVE = "f32sr"


def serving_block(n_plain: int):
    """1000-request Poisson trace (200/s) served with continuous batching (the
    quantum chosen on a 200-request prefix) vs the first n_plain requests run
    one at a time in arrival order; the stored oracle sample of served
    requests; the sustainable rate from a sweep of offered rates."""
    import numpy as np
    from paper_1510_08886_amd import serve
    from tests.golden.converged import SERVE, load_converged, rel_err_at
    cfg = wl.SERVE

    def trace_at(rate, n=cfg["requests"]):
        return wl.serve_trace(n, seed=cfg["seed"], rate=rate)

    trace = trace_at(cfg["rate"])
    kw = dict(storage=STORAGE_SERVE, tol=cfg["tol"], check_every=cfg["check_every"])
    quantum, q_rows = serve.tune_quantum(trace[:200], **kw)
    s = serve.serve(trace, quantum=quantum, **kw)
    lat = s["latency_s"]
    first = trace[:n_plain]
    sp = serve.serve(first, quantum=quantum, **kw)
    p = serve.serve_plain_fifo(first, **kw)
    same = all(a["steps"] == b["steps"] and abs(a["mdot"] - b["mdot"]) <= 1e-13 * abs(b["mdot"])
               for a, b in zip(sp["results"], p["results"]))
    span = max(r["t_done"] for r in s["results"]) - trace[0]["t"]
    gold = load_converged(SERVE) if SERVE.exists() else {}
    by_id = {r["req_id"]: r for r in s["results"]}
    errs = []
    for k, g in gold.items():
        assert (trace[k]["ny"], trace[k]["kn"], trace[k]["dvm"]) == (g["ny"], g["kn"], g["dvm"])
        errs.append(rel_err_at(g, by_id[k]["steps"], by_id[k]["mdot"]))
    sustainable, rows = serve.rate_sweep(lambda r: trace_at(r, 800), (200, 300, 400, 800),
                                         quantum=quantum, **kw)
    return {
        "workload": "1000 requests, Poisson 200/s, Ny~U[16,1024], Kn log-uniform [0.01,1], "
                    "DVM in {D2V17, D2V37}, tol 1e-8",
        "storage": "f32sr (FP32 deviations, FP64 collision, stochastic rounding)",
        "quantum": quantum,
        "quantum_trials": q_rows,
        "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
        "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
        "solves_per_s": round(len(trace) / span, 2),
        "wall_s": round(s["wall_s"], 3),
        "launches": s["launches"],
        "max_resident": s["max_active"],
        "mdot_rel_err_vs_oracle": dict(_err_stats(errs),
                                       note="stored FP64 oracle sample of the trace, at each "
                                            "served request's own stop step"),
        "sustainable_rate_per_s": sustainable,
        "rate_sweep": {"requests": 800, "rows": rows},
        "prefix": {"requests": n_plain,
                   "served_p50_s": round(float(np.percentile(sp["latency_s"], 50)), 4),
                   "served_p99_s": round(float(np.percentile(sp["latency_s"], 99)), 4),
                   "plain_p50_s": round(float(np.percentile(p["latency_s"], 50)), 4),
                   "plain_p99_s": round(float(np.percentile(p["latency_s"], 99)), 4),
                   "plain_solves_per_s": round(n_plain / p["busy_s"], 2),
                   "served_equals_plain": bool(same)},
    }


def channel_block():
    """The FP64 D2V17 channel, nx = 1, ny = 40, Kn = 0.1, 20000 steps from rest:
    launch-bound, so the figure is the time to solution; mass flow and profile
    against the stored FP64 oracle run of the same channel."""
    import numpy as np
    import torch

    from paper_1510_08886_amd import lbm

    c = wl.CHANNEL_D2V17
    rows = [l.split() for l in (ROOT / "tests" / "golden" / "channel_d2v17.txt").read_text()
            .splitlines() if l and not l.startswith("#")]
    gold = {r[0]: float(r[1]) for r in rows if r[0] != "ux"}
    ux_gold = np.array([float(r[2]) for r in rows if r[0] == "ux"])
    d = lbm.Dvm.named(c["dvm"])
    prob = lbm.Problem(dim=2, nx=c["nx"], ny=c["ny"], kn=c["kn"], ma=c["ma"], hermite_order=c["N"],
                       storage=c["storage"])
    s = lbm.Solver(d, prob, device="cuda:0").init()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    s.run(c["steps"])
    e1.record(s.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ob = s.observe()
    ux = ob["u"][:, 0, 0].cpu().numpy()
    s.close()
    return {"workload": "D2V17 N=3 FP64 channel 1x40, Kn=0.1, Ma=1e-3, from rest, "
                        f"{c['steps']} steps",
            "time_to_solution_s": round(ms * 1e-3, 4),
            "us_per_step": round(ms * 1e3 / c["steps"], 2),
            "mdot": ob["mdot"],
            "mdot_rel_err_vs_oracle": abs(ob["mdot"] - gold["mdot"]) / abs(gold["mdot"]),
            "u_max_rel_err_vs_oracle": float(np.max(np.abs(ux - ux_gold)) / np.max(np.abs(ux_gold)))}


def one_step_block(d, steps: int, warmup: int):
    """The headline channel stepped one lattice update per launch on one
    155 MB array updated in place (the two alternating in-place kinds of
    k_step2d): MLUPS and its HBM fraction at 2 V s bytes per update. The array
    fits the 256 MB last-level cache and consecutive steps reuse the L2."""
    import torch

    from paper_1510_08886_amd import lbm

    c = wl.THROUGHPUT_D2V37
    prob = lbm.Problem(dim=2, nx=c["nx"], ny=c["ny"], kn=c["kn"], ma=c["ma"], hermite_order=c["N"],
                       storage="f32", layout="in_place")
    s = lbm.Solver(d, prob, device="cuda:0")
    s.init(torch.from_numpy(wl.density_field(c["ny"], c["nx"], seed=c["seed"], amp=c["amp"])))
    s.run(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    s.run(steps)
    e1.record(s.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    mdot = s.mdot()
    s.close()
    nodes = c["nx"] * c["ny"]
    per_step = 2 * d.V * 4 * nodes
    gbs = per_step / (ms * 1e-3) / 1e9
    rec = profile_record(TRAFFIC_FILE)
    roof = {"bound": "hbm (array resident in the 256 MB LLC)", "achieved": round(gbs, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
            "bytes_per_launch": per_step, "llc_resident": True,
            "source": "HIP events over the timed steps",
            "achieved_hip_events": round(gbs, 1), "frac_hip_events": round(gbs / HBM_PEAK_GBS, 4),
            "traffic": None if rec is None else rec["bytes_per_launch"]}
    if rec is not None:
        kinds = rec["trace_ns_per_launch"]        # the two alternating in-place kinds
        tr_gbs = per_step / (sum(kinds.values()) / len(kinds) * 1e-9) / 1e9
        roof.update(achieved=round(tr_gbs, 1), frac=round(tr_gbs / HBM_PEAK_GBS, 4),
                    source="kernel trace " + rec["profile"] + " (mean duration per step)",
                    frac_kernel_trace=round(rec["trace_frac"], 4), profile=rec["profile"])
    return {"workload": "the headline channel, one array of 155 MB stepped in place, one step "
                        "per launch", "steps": steps,
            "mlups": round(nodes / (ms * 1e-3) / 1e6, 1), "ms_per_step": ms,
            "roofline": roof, "mdot": mdot}


def above_llc_block(steps: int = 1000):
    """The D2V37 FP32 channel at 4096 x 2048 (1.24 GB per population copy,
    above the 256 MB last-level cache), same physics, seeded density recipe
    and step count (1000) as the headline: the default layout there is two
    copies stepped ping-pong, two steps per launch. MLUPS and the HBM fraction
    of the two-step kernel against its own bytes model, next to a plain copy
    of one copy. (From the seeded random density the first ~100 steps of this
    kernel run slower than the rest, 320 falling to 270 us per step; from a
    uniform start it runs at the steady rate at once. The figure is the mean
    over the 1000 steps.)"""
    import torch

    from paper_1510_08886_amd import lbm

    c = wl.THROUGHPUT_D2V37
    nx, ny = 4096, 2048
    d = lbm.Dvm.named(c["dvm"])
    prob = lbm.Problem(dim=2, nx=nx, ny=ny, kn=c["kn"], ma=c["ma"], hermite_order=c["N"],
                       storage="f32")
    pop_bytes, _ = lbm.state_bytes(d, prob)
    s = lbm.Solver(d, prob, device="cuda:0")
    s.init(torch.from_numpy(wl.density_field(ny, nx, seed=c["seed"], amp=c["amp"])))
    s.run(6)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    s.run(steps)
    e1.record(s.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    mdot = s.mdot()
    s.close()
    nodes = nx * ny
    # the library steps this problem two steps per launch (k_pair2d): one
    # launch reads each population once and writes it once
    per_launch = 2 * d.V * 4 * nodes
    launch_s = 2 * ms * 1e-3
    gbs = per_launch / launch_s / 1e9
    single_model_gbs = 2 * d.V * 4 * nodes / (ms * 1e-3) / 1e9
    cg = copy_gbs(per_launch // 2)
    rec = profile_record(PAIR_TRAFFIC_FILE)
    roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_launch": per_launch,
            "model": "two steps per launch: each population read once and written once per "
                     "launch, 148 B per lattice update",
            "source": "HIP events over the timed launches",
            "achieved_hip_events": round(gbs, 1), "frac_hip_events": round(gbs / HBM_PEAK_GBS, 4),
            "traffic": None if rec is None else rec["bytes_per_launch"]}
    if rec is not None:
        tr_gbs = per_launch / (rec["trace_ns_per_launch"] * 1e-9) / 1e9
        roof.update(achieved=round(tr_gbs, 1), frac=round(tr_gbs / HBM_PEAK_GBS, 4),
                    source="kernel trace " + rec["profile"] + " (mean duration per launch)",
                    frac_kernel_trace=round(rec["trace_frac"], 4), profile=rec["profile"])
    return {"workload": "D2V37 FP32 Poiseuille channel 4096x2048, Kn=0.05, N=4, seeded "
                        "rho=1+1e-3*N(0,1); ping-pong copies of 1.24 GB (above the LLC), "
                        "two steps per launch",
            "population_bytes": pop_bytes, "steps": steps,
            "mlups": round(nodes / (ms * 1e-3) / 1e6, 1), "ms_per_step": ms,
            "roofline": roof,
            "single_step_model_gbs": round(single_model_gbs, 1),
            "copy_gbs": round(cg, 1), "mdot": mdot}


def duct_block():
    """3D square duct on D3V39, 128 x 256 x 256 (periodic x, diffuse Maxwell
    walls on the four y and z faces), Kn = 0.1, from rest, 500 steps with FP32
    and FP16-deviation populations; mass-flow error against the FP64 oracle's
    streamwise-invariant (one x column) run of the same duct, stored under
    tests/golden/ by a script that calls only the oracle."""
    import torch

    from paper_1510_08886_amd import lbm

    c = wl.DUCT_D3V39
    gold = {}
    for line in (ROOT / "tests" / "golden" / "duct_d3v39_mdot.txt").read_text().splitlines():
        if line and not line.startswith("#"):
            t = line.split()
            gold[int(t[0])] = float(t[1])
    want = gold[c["steps"]]
    d = lbm.Dvm.named(c["dvm"])
    nodes = c["nx"] * c["ny"] * c["nz"]
    out = {"workload": "D3V39 N=3 square duct 128x256x256, Kn=0.1, Ma=1e-3, from rest, "
                       f"{c['steps']} steps", "oracle_mdot": want}
    copy = {size: copy_gbs(d.V * size * nodes) for size in (4, 2)}
    for storage, size in (("f32", 4), ("f16dev", 2)):
        prob = lbm.Problem(dim=3, nx=c["nx"], ny=c["ny"], nz=c["nz"], kn=c["kn"], ma=c["ma"],
                           hermite_order=c["N"], storage=storage)
        s = lbm.Solver(d, prob, device="cuda:0").init()
        # untimed warm-up steps (page tables, caches), then the same solve from
        # rest again: init resets the state and the step counter, so the timed
        # 500 steps are bit for bit those of a fresh solver
        s.run(5)
        s.init()
        m0 = s.observe()["mass"]
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s.stream)
        s.run(c["steps"])
        e1.record(s.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        ob = s.observe()
        gbs = 2 * d.V * size * nodes / (ms * 1e-3 / c["steps"]) / 1e9
        out[storage] = {"mlups": round(nodes * c["steps"] / (ms * 1e-3) / 1e6, 1),
                        "ms_per_step": ms / c["steps"],
                        "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                        "copy_gbs": round(copy[size], 1),
                        "frac_of_copy": round(gbs / copy[size], 4),
                        "mdot": ob["mdot"],
                        "mdot_rel_err_vs_oracle": abs(ob["mdot"] - want) / abs(want),
                        "mass_drift": abs(ob["mass"] - m0) / m0}
        s.close()
    return out


def scattering_block():
    """Scattering stencils (no velocity parallel to the walls): the D2V32
    channel at 2048 x 512 (halo 12) and the D3V96 duct at 128 x 256 x 256
    (halo 7), FP32 populations, from the seeded density field / rest. MLUPS and
    the HBM fraction of the step kernel (algorithmic bytes 2 V 4 per update)."""
    import torch

    from paper_1510_08886_amd import lbm

    out = {}
    for key, c in (("d2v32_channel", wl.SCATTER_D2V32), ("d3v96_duct", wl.SCATTER_D3V96)):
        d = lbm.Dvm.named(c["dvm"])
        dim = lbm.NAMED_DVMS[c["dvm"]]["dim"]
        nz = c.get("nz", 1)
        prob = lbm.Problem(dim=dim, nx=c["nx"], ny=c["ny"], nz=nz, kn=c["kn"], ma=c["ma"],
                           hermite_order=c["N"], storage="f32")
        s = lbm.Solver(d, prob, device="cuda:0")
        nodes = c["nx"] * c["ny"] * nz
        if dim == 2:
            s.init(torch.from_numpy(wl.density_field(c["ny"], c["nx"])))
        else:
            s.init()
        s.run(5)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s.stream)
        s.run(c["steps"])
        e1.record(s.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        gbs = 2 * d.V * 4 * nodes / (ms * 1e-3 / c["steps"]) / 1e9
        pop_bytes = lbm.state_bytes(d, prob)[0]
        out[key] = {"V": d.V, "nodes": nodes, "steps": c["steps"],
                    "mlups": round(nodes * c["steps"] / (ms * 1e-3) / 1e6, 1),
                    "ms_per_step": ms / c["steps"], "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                    "population_bytes": pop_bytes, "llc_resident": pop_bytes <= LLC_BYTES,
                    "mdot": s.mdot()}
        s.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=wl.THROUGHPUT_D2V37["steps"])
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched Kn sweep")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving trace")
    ap.add_argument("--no-duct", action="store_true", help="skip the 3D duct runs")
    ap.add_argument("--no-channel", action="store_true", help="skip the FP64 D2V17 channel run")
    ap.add_argument("--no-scatter", action="store_true", help="skip the scattering-stencil runs")
    ap.add_argument("--no-parity", action="store_true",
                    help="skip the untimed 1000-step run of the headline against the oracle golden")
    ap.add_argument("--no-above-llc", action="store_true",
                    help="skip the 4096 x 2048 channel whose copies exceed the last-level cache")
    ap.add_argument("--plain-serve-requests", type=int, default=100,
                    help="prefix of the serving trace run by the one-at-a-time plain baseline")
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
    bytes_per_step = 2 * d.V * 4 * nodes           # each population read once, written once
    achieved = bytes_per_step / (ms * 1e-3 / args.steps) / 1e9
    obs = s.observe()
    # stability: five more timed blocks of the same length after the timed
    # region (not part of value)
    reps = []
    for _ in range(5):
        e0.record(stream)
        s.run(args.steps)
        e1.record(stream)
        torch.cuda.synchronize()
        reps.append(e0.elapsed_time(e1) / args.steps)
    s.close()
    parity = None if args.no_parity else throughput_parity(d, prob)
    rec = profile_record(HEAD_TRAFFIC_FILE)
    # the library steps this channel two lattice updates per launch (k_pair2d);
    # the algorithmic bytes are those of two updates, 2 V s each
    algo_per_launch = 2 * bytes_per_step
    roofline = {"bound": "hbm", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if rec is None else rec["bytes_per_launch"],
                "bytes_per_launch": algo_per_launch,
                "model": "algorithmic 2 V s = 296 B per lattice update (each population read "
                         "once and written once per update); one launch of k_pair2d advances "
                         "two updates and keeps the intermediate one in LDS, so the HBM bytes "
                         "it moves (traffic, counters) are about half of these",
                "llc_resident": False, "source": "HIP events over the timed steps",
                "achieved_hip_events": round(achieved, 1),
                "frac_hip_events": round(achieved / HBM_PEAK_GBS, 4),
                "note": "two ping-pong copies of 155 MB (310 MB, above the 256 MB last-level "
                        "cache), two steps per launch; one_step_in_place holds the single-step "
                        "kernels on one 155 MB array"}
    if rec is not None:
        tr_ns = rec["trace_ns_per_launch"]
        tr_gbs = algo_per_launch / (tr_ns * 1e-9) / 1e9
        moved = rec["bytes_per_launch"] / (tr_ns * 1e-9) / 1e9
        roofline.update(achieved=round(tr_gbs, 1), frac=round(tr_gbs / HBM_PEAK_GBS, 4),
                        source="kernel trace " + rec["profile"] + " (mean duration per launch)",
                        frac_kernel_trace=round(rec["trace_frac"], 4), profile=rec["profile"],
                        moved_gbs=round(moved, 1), moved_frac=round(moved / HBM_PEAK_GBS, 4))
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
        "roofline": roofline,
        "wall_s": round(wall, 3),
        "repeat_ms_per_step": {"blocks": [round(x, 5) for x in reps],
                               "median": round(sorted(reps)[2], 5),
                               "note": "five more blocks of the same step count after the "
                                       "timed region (HIP events), for its spread"},
        "mdot_after": obs["mdot"],
        "parity_vs_oracle": parity,
    }
    cg = copy_gbs(bytes_per_step // 2)
    out["measured_copy"] = {"bytes_each_way": bytes_per_step // 2, "gbs": round(cg, 1),
                            "step_frac_of_copy": round(achieved / cg, 4),
                            "note": "plain streaming copy of one population array (lbm_stream_copy); "
                                    "step_frac_of_copy compares the algorithmic bytes per step"}
    out["one_step_in_place"] = one_step_block(d, args.steps, args.warmup)
    if not args.no_above_llc:
        out["above_llc"] = above_llc_block()
    if not args.no_batch:
        out["batched"] = batched_block()
    if not args.no_serve:
        out["serving"] = serving_block(args.plain_serve_requests)
    if not args.no_channel:
        out["channel_d2v17_f64"] = channel_block()
    if not args.no_duct:
        out["duct"] = duct_block()
    if not args.no_scatter:
        out["scattering"] = scattering_block()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
