"""Graph replay of step sequences (lbm_run on small problems): a solver that
replays captured HIP graphs against one that launches every step, bit for bit,
over chunks of odd and even lengths with eager work and synchronisations between
them, so cached graphs are replayed many times from each starting state."""
import numpy as np
import pytest

import lbm_workloads as wl

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

CHUNKS = [1, 7, 2, 33, 100, 3, 64, 64, 17]


def _pair(name, N, nx, ny, nz=1, storage="f32", graph=16, ma=1e-2, seed=1):
    from paper_1510_08886_amd import lbm
    d = lbm.Dvm.named(name)
    dim = lbm.NAMED_DVMS[name]["dim"]
    prob = lbm.Problem(dim=dim, nx=nx, ny=ny, nz=nz, kn=0.1, ma=ma, hermite_order=N,
                       storage=storage)
    nodes = nx * ny * nz
    rho, u = wl.random_state(nodes, dim, seed=seed, amp=1e-2)
    out = []
    for g in (graph, 0):
        s = lbm.Solver(d, prob)
        s.set_graph_steps(g)
        s.init(torch.from_numpy(rho), torch.from_numpy(u))
        out.append(s)
    return out


@pytest.mark.parametrize("name,N,nx,ny,nz,storage", [
    ("D2V17", 3, 1, 40, 1, "f64"),     # the launch-bound FP64 channel
    ("D2V37", 4, 70, 13, 1, "f32"),    # in place, ragged tiles
    ("D2V37", 4, 128, 20, 1, "f32"),   # aligned rows, per-XCD tile bands
    ("D3V39", 3, 20, 16, 14, "f32"),   # duct
])
def test_graph_replay_matches_one_launch_per_step(name, N, nx, ny, nz, storage):
    a, b = _pair(name, N, nx, ny, nz, storage)
    for k, n in enumerate(CHUNKS):
        a.run(n)
        b.run(n)
        assert a.steps == b.steps
        assert torch.equal(a.export(), b.export()), (k, n)
        if k % 3 == 1:                      # eager work between replays
            assert a.observe()["mdot"] == b.observe()["mdot"]
    # a fresh start from the same solver reuses the cached graphs
    a.init()
    b.init()
    a.run(40)
    b.run(40)
    assert torch.equal(a.export(), b.export())
    # checkpoint resume in between
    ck = a.export().clone()
    a.import_(ck)
    b.import_(ck)
    a.run(21)
    b.run(21)
    assert torch.equal(a.export(), b.export())
    a.close()
    b.close()


def test_graph_replay_default_and_fp16():
    from paper_1510_08886_amd import lbm
    d = lbm.Dvm.named("D2V37")
    prob = lbm.Problem(dim=2, nx=64, ny=12, kn=0.1, hermite_order=4, storage="f16dev")
    s = lbm.Solver(d, prob).init()
    with pytest.raises(lbm.LbmError):
        s.set_graph_steps(8)       # stochastic rounding keys on the step counter
    s.set_graph_steps(0)
    s.run(10)
    s.close()


def test_graph_replay_ping_pong_path():
    """Graphs switched on for a ping-pong solver (a 550 MB FP64 duct copy): the
    two buffers swap every step, so a replay must start from the same pair."""
    a, b = _pair("D3V39", 3, 64, 166, 166, "f64", graph=4)
    for n in (3, 4, 5, 8, 1):
        a.run(n)
        b.run(n)
        assert torch.equal(a.export(), b.export()), n
    a.close()
    b.close()
