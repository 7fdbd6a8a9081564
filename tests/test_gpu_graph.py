"""Multi-step launches of lbm_run on small problems, against a solver that
launches every step, bit for bit, over chunks of odd and even lengths with eager
work and synchronisations between them:

* graph replay (captured HIP graphs, cached and replayed many times from each
  starting state);
* resident stepping (one workgroup loops over the steps of a 2D in-place
  problem of at most 256 nodes, FP16 stochastic rounding included)."""
import numpy as np
import pytest

import lbm_workloads as wl

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

CHUNKS = [1, 7, 2, 33, 100, 3, 64, 64, 17]


def _pair(name, N, nx, ny, nz=1, storage="f32", graph=16, ma=1e-2, seed=1, resident=0):
    from paper_1510_08886_amd import lbm
    d = lbm.Dvm.named(name)
    dim = lbm.NAMED_DVMS[name]["dim"]
    prob = lbm.Problem(dim=dim, nx=nx, ny=ny, nz=nz, kn=0.1, ma=ma, hermite_order=N,
                       storage=storage)
    nodes = nx * ny * nz
    rho, u = wl.random_state(nodes, dim, seed=seed, amp=1e-2)
    out = []
    for g, r in ((graph, resident), (0, 0)):
        s = lbm.Solver(d, prob)
        if dim == 2 and nodes <= 256:
            s.set_resident_steps(r)
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


@pytest.mark.parametrize("storage", ["f16dev", "f32sr"])
def test_graph_replay_default_and_fp16(storage):
    from paper_1510_08886_amd import lbm
    d = lbm.Dvm.named("D2V37")
    prob = lbm.Problem(dim=2, nx=64, ny=12, kn=0.1, hermite_order=4, storage=storage)
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


def test_graph_cache_eviction_and_teardown_in_flight():
    """More distinct step sequences than the solver caches graphs for (8): the
    oldest graphs are destroyed while later replays are queued, and solvers are
    destroyed with replays still in flight; every result stays equal to one
    launch per step, and a solver created after the teardown steps correctly."""
    a, b = _pair("D2V17", 3, 1, 300, storage="f64", graph=64)
    for n in (2, 4, 6, 8, 10, 12, 14, 16, 18, 20, 2, 4, 22, 64, 130):
        a.run(n)
        b.run(n)
    assert torch.equal(a.export(), b.export())
    # teardown with replays queued behind a long sequence
    a.run(640)
    a.close()
    b.close()
    c, d = _pair("D2V17", 3, 1, 300, storage="f64", graph=64)
    c.run(300)
    d.run(300)
    assert torch.equal(c.export(), d.export())
    c.close()
    d.close()


@pytest.mark.parametrize("name,N,nx,ny,storage", [
    ("D2V17", 3, 1, 40, "f64"),      # the launch-bound FP64 channel
    ("D2V37", 4, 20, 12, "f32"),     # 240 nodes, wall rows on both sides
    ("D2V37", 4, 16, 16, "f16dev"),  # 256 nodes; stochastic rounding numbered per step
    ("D2V17", 3, 1, 40, "f32sr"),    # FP64 collision, FP32 stochastic rounding per step
    ("D2V37", 5, 1, 21, "f32"),      # Hermite order 5 variant
    ("D2V32", 4, 5, 29, "f64"),      # halo 12, periodic wraps
])
def test_resident_stepping_matches_one_launch_per_step(name, N, nx, ny, storage):
    a, b = _pair(name, N, nx, ny, 1, storage, graph=0, resident=50)
    for k, n in enumerate(CHUNKS):
        a.run(n)
        b.run(n)
        assert a.steps == b.steps
        assert torch.equal(a.export(), b.export()), (k, n)
        if k % 3 == 1:
            assert a.observe()["mdot"] == b.observe()["mdot"]
    ck = a.export().clone()
    a.import_(ck)
    b.import_(ck)
    a.run(33)
    b.run(33)
    assert torch.equal(a.export(), b.export())
    a.close()
    b.close()


def test_resident_stepping_default_and_limits():
    from paper_1510_08886_amd import lbm
    d = lbm.Dvm.named("D2V17")
    big = lbm.Solver(d, lbm.Problem(dim=2, nx=17, ny=16, kn=0.1, hermite_order=3)).init()
    with pytest.raises(lbm.LbmError):
        big.set_resident_steps(8)      # 272 nodes: more than one node per thread
    big.close()
    d3 = lbm.Dvm.named("D3V39")
    duct = lbm.Solver(d3, lbm.Problem(dim=3, nx=2, ny=8, nz=8, kn=0.1, hermite_order=3)).init()
    with pytest.raises(lbm.LbmError):
        duct.set_resident_steps(8)
    duct.close()
