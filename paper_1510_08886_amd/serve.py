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
                  max_steps=2_000_000, autotune=True, trial_steps=200, pool_bytes=256 << 20,
                  tuning=None):
    """All channels in one persistent launch. max_steps is one cap or a list
    with one cap per channel. With autotune the workgroup size, resident
    workgroups per CU and work-queue order are chosen by timed trials
    (lbm_batch_autotune; the timed run then replays the graph captured by the
    winning trial); otherwise `tuning` (a dict of lbm.Batch.tune arguments)
    or the defaults apply. Returns results in request order, the makespan (s),
    the tuning used and the engine's counters."""
    import torch

    d = lbm.Dvm.named(dvm_name)
    N = lbm.NAMED_DVMS[dvm_name]["N"]
    b = lbm.Batch(max(1, len(channels)), storage=storage, pool_bytes=pool_bytes)

    caps = list(max_steps) if np.ndim(max_steps) else [max_steps] * len(channels)
    for k, ch in enumerate(channels):
        b.submit(d, ch["ny"], ch["kn"], N=N, tol=tol, check_every=check_every,
                 max_steps=int(caps[k]), req_id=k)
    tune_s = 0.0
    chosen = None
    if autotune:
        t0 = time.perf_counter()
        chosen = b.autotune(trial_steps)
        tune_s = time.perf_counter() - t0
    elif tuning:
        b.tune(**tuning)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = b.run_persistent()
    torch.cuda.synchronize()
    makespan = time.perf_counter() - t0
    res.sort(key=lambda r: r["req_id"])
    st = b.stats()
    b.close()
    if chosen is None:
        chosen = dict(threads=st["threads"], slots_per_cu=st["slots_per_cu"],
                      order=lbm.BATCH_ORDERS[st["order"]])
    return dict(results=res, makespan_s=makespan, threads=st["threads"], tuning=chosen,
                tune_s=tune_s, graph_replays=st["graph_replays"], launches=st["launches"])


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
                launches=stats["launches"], max_active=max_active, quantum=quantum,
                threads=threads)


def tune_quantum(trace, candidates=(250, 500, 1000, 2000), **kw):
    """Serve `trace` (a short prefix of the real one) once per candidate
    quantum (steps per served launch) and return the quantum with the lowest
    p99 latency, with every candidate's p50 / p99 (s)."""
    out = {}
    for q in candidates:
        r = serve(trace, quantum=q, **kw)
        out[q] = (float(np.percentile(r["latency_s"], 50)), float(np.percentile(r["latency_s"], 99)))
    best = min(out, key=lambda q: out[q][1])
    return best, {str(q): {"p50_s": round(v[0], 4), "p99_s": round(v[1], 4)} for q, v in out.items()}


def rate_sweep(make_trace, rates, **kw):
    """Serve a trace at each offered Poisson rate (make_trace(rate) -> trace).
    Per rate: p50 / p90 / p99 latency, the arrival and completion rates in the
    middle half of the trace (the n/2 arrivals and the completions between the
    arrivals of requests n/4 and 3n/4, over that span: equal when the engine
    keeps up, the completions at its capacity when it does not; the ends are
    left out because the trace starts empty and its last long solves drain
    after the arrivals stop) and the drift of the tail, p90 latency of the
    second half of the trace (by arrival) over that of the first half. A rate
    is sustained when the middle half completes at least 90 % of its arrivals
    and the tail drifts up by at most 50 %: a queue that grows over the trace
    fails both. The sustainable rate is the largest rate sustained together
    with every lower one."""
    rows = []
    for rate in rates:
        tr = make_trace(rate)
        r = serve(tr, **kw)
        lat = r["latency_s"]
        n = len(lat)
        h = n // 2
        ta, tb = tr[n // 4]["t"], tr[3 * n // 4]["t"]
        t_done = np.array([x["t_done"] for x in r["results"]])
        arrived = 3 * n // 4 - n // 4
        completed = int(np.sum((t_done >= ta) & (t_done < tb)))
        span = max(tb - ta, 1e-9)
        drift = float(np.percentile(lat[h:], 90) / max(np.percentile(lat[:h], 90), 1e-9))
        rows.append({"rate": rate, "p50_s": round(float(np.percentile(lat, 50)), 4),
                     "p90_s": round(float(np.percentile(lat, 90)), 4),
                     "p99_s": round(float(np.percentile(lat, 99)), 4),
                     "arrived_per_s": round(arrived / span, 2),
                     "completed_per_s": round(completed / span, 2), "p90_drift": round(drift, 3),
                     "max_resident": r["max_active"],
                     "sustained": bool(completed >= 0.9 * arrived and drift <= 1.5)})
    sustainable = None
    for row in rows:
        if not row["sustained"]:
            break
        sustainable = row["rate"]
    return sustainable, rows


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
