"""Host logic of the serving measurements (no GPU): the sustained-rate test of
serve.rate_sweep and the quantum choice of serve.tune_quantum, on a stand-in
for the served engine whose completion times follow a single-server queue."""
import numpy as np

from paper_1510_08886_amd import serve


def _trace(rate, n=400, seed=3):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    return [dict(id=k, t=float(t[k]), ny=32, kn=0.1, dvm="D2V17") for k in range(n)]


def _fake_serve(capacity):
    """FIFO server finishing one request every 1/capacity seconds."""
    def run(tr, **kw):
        clock = 0.0
        res = []
        for r in tr:
            clock = max(clock, r["t"]) + 1.0 / capacity
            res.append(dict(req_id=r["id"], t_done=clock))
        lat = np.array([x["t_done"] - r["t"] for x, r in zip(res, tr)])
        return dict(results=res, latency_s=lat, max_active=1, quantum=kw.get("quantum", 1000))
    return run


def test_rate_sweep_finds_the_capacity(monkeypatch):
    monkeypatch.setattr(serve, "serve", _fake_serve(capacity=500.0))
    best, rows = serve.rate_sweep(_trace, (100, 200, 400, 800, 1600))
    flags = {r["rate"]: r["sustained"] for r in rows}
    assert flags == {100: True, 200: True, 400: True, 800: False, 1600: False}
    assert best == 400
    over = [r for r in rows if r["rate"] == 1600][0]
    assert abs(over["completed_per_s"] - 500.0) < 25     # capacity, not the offered rate
    assert over["p90_drift"] > 1.5                       # the queue grows


def test_rate_sweep_stops_at_the_first_failure(monkeypatch):
    monkeypatch.setattr(serve, "serve", _fake_serve(capacity=150.0))
    best, rows = serve.rate_sweep(_trace, (100, 200, 120))
    assert [r["sustained"] for r in rows] == [True, False, True]
    assert best == 100


def test_tune_quantum_picks_lowest_p99(monkeypatch):
    def fake(tr, quantum=1000, **kw):
        lat = np.full(len(tr), 1.0 + abs(quantum - 700) / 1000.0)
        return dict(results=[], latency_s=lat)
    monkeypatch.setattr(serve, "serve", fake)
    best, rows = serve.tune_quantum(_trace(100, n=20), candidates=(250, 500, 1000, 2000))
    assert best == 500 and set(rows) == {"250", "500", "1000", "2000"}
