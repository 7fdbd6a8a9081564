"""Batched Kn sweeps and a serving loop over the library's batch engine, and the
one-solve-at-a-time plain baselines they are compared with.

The physics of every solve is the plane Poiseuille channel of Section VI of the
paper (nx = 1, diffuse Maxwell walls, body force for Ma = 1e-3), run from rest
to a steady-state tolerance on the normalised mass flow (Eq. pf.1).
"""
from __future__ import annotations

import time

import numpy as np

from . import lbm


def _dvms(names):
    return {n: lbm.Dvm.named(n) for n in names}


def batched_sweep(channels, dvm_name="D2V37", storage="f32", tol=1e-8, check_every=100,
                  max_steps=2_000_000, autotune=True, trial_steps=200, pool_bytes=256 << 20):
    """All channels in one persistent launch (hipGraph). max_steps is one cap
    or a list with one cap per channel. Returns results in request order, the
    makespan (s) and the workgroup size used."""
    import torch

    d = lbm.Dvm.named(dvm_name)
    N = lbm.NAMED_DVMS[dvm_name]["N"]
    b = lbm.Batch(max(1, len(channels)), storage=storage, pool_bytes=pool_bytes)

    caps = list(max_steps) if np.ndim(max_steps) else [max_steps] * len(channels)

    def submit_all(cap):
        for k, ch in enumerate(channels):
            b.submit(d, ch["ny"], ch["kn"], N=N, tol=tol, check_every=check_every,
                     max_steps=int(min(caps[k], cap)), req_id=k)

    threads = None
    tune_s = 0.0
    submit_all(max(caps))
    if autotune:
        t0 = time.perf_counter()
        threads = b.autotune(trial_steps)
        tune_s = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = b.run_persistent()
    torch.cuda.synchronize()
    makespan = time.perf_counter() - t0
    res.sort(key=lambda r: r["req_id"])
    st = b.stats()
    b.close()
    return dict(results=res, makespan_s=makespan, threads=threads or st["threads"], tune_s=tune_s)


def plain_sweep(channels, dvm_name="D2V37", storage="f32", tol=1e-8, check_every=100,
                max_steps=2_000_000, budget_s=None):
    """The same channels one at a time through the single-solve path
    (lbm_run_to_tol, a mass-flow check every check_every steps): channels of
    at most 256 rows step in one-workgroup resident launches of many steps,
    larger ones replay captured graphs of up to 256 step launches. Optionally
    stop after budget_s seconds; returns the results done and their total
    time."""
    import torch

    d = lbm.Dvm.named(dvm_name)
    N = lbm.NAMED_DVMS[dvm_name]["N"]
    out = []
    total = 0.0
    for k, ch in enumerate(channels):
        prob = lbm.Problem(dim=2, nx=1, ny=ch["ny"], kn=ch["kn"], hermite_order=N, storage=storage)
        s = lbm.Solver(d, prob).init()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.run_to_tol(tol=tol, check_every=check_every, max_steps=max_steps)
        dt = time.perf_counter() - t0
        total += dt
        out.append(dict(req_id=k, steps=r["steps"], mdot=r["mdot"],
                        status="converged" if r["converged"] else "not_converged", seconds=dt))
        s.close()
        if budget_s is not None and total > budget_s:
            break
    return dict(results=out, total_s=total)


def serve(trace, storage="f32", tol=1e-8, check_every=100, max_steps=2_000_000, max_slots=256,
          quantum=1000, threads=512, pool_bytes=1 << 30, idle_sleep=2e-4):
    """Real-time serving loop: each request is submitted at its arrival time
    (seconds after the start) and admitted by the engine when a slot and pool
    memory are free; returns per-request latency (completion - arrival)."""
    dv = _dvms(sorted({r["dvm"] for r in trace}))
    b = lbm.Batch(max_slots, storage=storage, pool_bytes=pool_bytes)
    b.tune(threads, quantum)
    n = len(trace)
    done = {}
    i = 0
    max_active = 0
    t0 = time.perf_counter()
    while len(done) < n:
        now = time.perf_counter() - t0
        while i < n and trace[i]["t"] <= now:
            r = trace[i]
            b.submit(dv[r["dvm"]], r["ny"], r["kn"], N=lbm.NAMED_DVMS[r["dvm"]]["N"], tol=tol,
                     check_every=check_every, max_steps=max_steps, req_id=r["id"])
            i += 1
        got = b.poll()
        tnow = time.perf_counter() - t0
        for g in got:
            done[g["req_id"]] = dict(g, t_done=tnow)
        st = b.stats()
        max_active = max(max_active, st["active"])
        if not got and (i >= n or trace[i]["t"] > tnow + idle_sleep):
            time.sleep(idle_sleep)
    wall = time.perf_counter() - t0
    lat = np.array([done[r["id"]]["t_done"] - r["t"] for r in trace])
    stats = b.stats()
    b.close()
    return dict(results=[done[r["id"]] for r in trace], latency_s=lat, wall_s=wall,
                launches=stats["launches"], max_active=max_active)


def serve_plain_fifo(trace, storage="f32", tol=1e-8, check_every=100, max_steps=2_000_000):
    """One solve at a time in arrival order. Durations are measured; the FIFO
    timeline is start_i = max(arrival_i, done_{i-1}), done_i = start_i + d_i."""
    dv = _dvms(sorted({r["dvm"] for r in trace}))
    import torch
    clock = 0.0
    out = []
    for r in trace:
        prob = lbm.Problem(dim=2, nx=1, ny=r["ny"], kn=r["kn"],
                           hermite_order=lbm.NAMED_DVMS[r["dvm"]]["N"], storage=storage)
        s = lbm.Solver(dv[r["dvm"]], prob).init()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = s.run_to_tol(tol=tol, check_every=check_every, max_steps=max_steps)
        dt = time.perf_counter() - t0
        s.close()
        start = max(clock, r["t"])
        clock = start + dt
        out.append(dict(req_id=r["id"], steps=res["steps"], mdot=res["mdot"], seconds=dt,
                        latency=clock - r["t"]))
    return dict(results=out, latency_s=np.array([o["latency"] for o in out]),
                busy_s=sum(o["seconds"] for o in out), makespan_s=clock - trace[0]["t"])
