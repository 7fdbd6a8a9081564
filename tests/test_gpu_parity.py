"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs. Bars: FP64 path <= 1e-12 relative on the velocity profile
and mass flow; FP32 storage <= 1e-5 relative on mass flow; FP16-deviation
storage <= 1e-3 relative on mass flow. FP32 storage of fbar itself (f32raw) is
measured against the same oracle and documented, not held to the FP32 bar: its
rounding step is ~6e-8 of w rho0, which is 3e-5 of the Ma = 1e-3 flow signal."""
import os

import numpy as np
import pytest

import lbm_workloads as wl
from tests.parity import make_pair, populations_both

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_08886_amd import lbm
    lbm.lib()


def _rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


def test_f64_channel_d2v17_full_run():
    """Plain FP64 Poiseuille channel on D2V17, Nx=1 x Ny=40, Kn=0.1, 20000 steps."""
    c = wl.CHANNEL_D2V17
    d, g, o = make_pair(c["dvm"], c["N"], c["nx"], c["ny"], kn=c["kn"], ma=c["ma"])
    g.run(c["steps"])
    o.run(c["steps"])
    og, oo = g.observe(), o.observe()
    ug = og["u"][..., 0].cpu().numpy()
    uo = oo["u"][..., 0]
    assert _rel(ug, uo) <= 1e-12
    assert abs(og["mdot"] - oo["mdot"]) <= 1e-12 * abs(oo["mdot"])
    assert abs(og["mass"] - oo["mass"]) <= 1e-13 * oo["mass"]
    pg, po = populations_both(d, g, o)
    assert np.max(np.abs(pg - po)) <= 1e-14


@pytest.mark.parametrize("name,N,nx,ny,steps", [
    ("D2V37", 4, 70, 13, 7),     # two x-tiles plus a ragged tail, rows span several waves
    ("D2V17", 3, 2, 5, 4),       # nx < |e_x|: periodic wrap of multi-speed shifts
    ("D2V17", 3, 4, 3, 3),       # ny = largest |e_y|: every row is a wall row
    ("D2V37", 3, 65, 6, 5),      # ny < 2 * halo: rows next to both walls
    ("D2V37", 4, 1, 21, 9),      # streamwise-invariant column
    ("D2V32", 4, 70, 12, 3),     # scattering stencil, |e| up to 12: every row a wall row
    ("D2V32", 3, 5, 29, 4),      # nx < |e_x| = 12 (multiple wraps), rows off both walls
])
def test_f64_random_state_elementwise(name, N, nx, ny, steps):
    rho, u = wl.random_state(nx * ny, 2, seed=nx * 131 + ny, amp=2e-2)
    d, g, o = make_pair(name, N, nx, ny, kn=0.07, ma=2e-2, rho=rho, u=u)
    pg, po = populations_both(d, g, o)
    assert np.max(np.abs(pg - po)) <= 1e-16
    g.run(steps)
    o.run(steps)
    pg, po = populations_both(d, g, o)
    assert np.max(np.abs(pg - po)) <= 1e-14
    og, oo = g.observe(), o.observe()
    np.testing.assert_allclose(og["rho"].cpu().numpy(), oo["rho"], rtol=1e-14)
    np.testing.assert_allclose(og["u"].cpu().numpy()[..., :2], oo["u"][..., :2], rtol=0, atol=1e-15)


@pytest.mark.parametrize("storage,tol_mdot,tol_pop", [("f32", 1e-5, 1e-8), ("f16dev", 1e-3, 1e-4),
                                                      ("f32raw", 1e-4, 1e-6), ("f32sr", 1e-6, 1e-8)])
def test_low_precision_storage(storage, tol_mdot, tol_pop):
    nx, ny = 130, 24
    rho = wl.density_field(ny, nx, seed=7, amp=1e-3)
    d, g, o = make_pair("D2V37", 4, nx, ny, kn=0.05, storage=storage, rho=rho)
    g.run(400)
    o.run(400)
    og, oo = g.observe(), o.observe()
    assert abs(og["mdot"] - oo["mdot"]) <= tol_mdot * abs(oo["mdot"])
    pg, po = populations_both(d, g, o)
    w = d.weights[:, None, None]
    assert np.max(np.abs(pg - po) / w) <= tol_pop


@pytest.mark.parametrize("nx,ny", [(128, 20), (512, 13), (192, 11), (64, 64)])
@pytest.mark.parametrize("storage,tol_mdot,tol_pop", [("f64", 1e-12, 1e-14), ("f32", 1e-5, 1e-8),
                                                      ("f16dev", 1e-3, 1e-4), ("f32sr", 1e-6, 1e-8)])
def test_aligned_rows_in_place(storage, tol_mdot, tol_pop, nx, ny):
    """Rows of whole 64-node blocks take the row-grid kernels (tiles of 128,
    256 and 64 nodes; 1, 2 and 3 tiles per row; the per-XCD tile bands end
    mid-row when the tile count is not a multiple of 8), in 16-bit storage with
    buffer addressing: both in-place kinds (odd and even step counts) element
    by element against the oracle. In the 64 x 64 channel each XCD band holds 8
    tiles, so the node-local kind's wall bands take their 3 wall tiles first
    and then run the other 5 in the opposite direction."""
    rho, u = wl.random_state(nx * ny, 2, seed=21 + nx + ny, amp=1e-3)
    d, g, o = make_pair("D2V37", 4, nx, ny, kn=0.05, storage=storage, rho=rho, u=u)
    w = d.weights[:, None, None]
    for steps in (1, 40, 59):
        g.run(steps)
        o.run(steps)
        pg, po = populations_both(d, g, o)
        assert np.max(np.abs(pg - po) / w) <= tol_pop, steps
    og, oo = g.observe(), o.observe()
    assert abs(og["mdot"] - oo["mdot"]) <= tol_mdot * abs(oo["mdot"])


@pytest.mark.parametrize("nx,ny", [(128, 30), (192, 13), (64, 120)])
@pytest.mark.parametrize("storage,tol_pop", [("f64", 1e-14), ("f32", 1e-8), ("f16dev", 1e-4)])
def test_aligned_rows_wide_stencil(storage, tol_pop, nx, ny):
    """The scattering stencil D2V32 (halo 12) on whole 64-node rows takes the
    buffer-addressed row-grid kernels in every storage: rows 12..17 of the
    30-row channel are off both walls, every row of the 13-row one is a wall
    row, and the 120-row one has XCD bands of 15 tiles whose first 12 (the
    wall rows) come first in the node-local kind. Both in-place kinds, element
    by element against the oracle."""
    rho, u = wl.random_state(nx * ny, 2, seed=5 + nx + ny, amp=1e-3)
    d, g, o = make_pair("D2V32", 4, nx, ny, kn=0.05, storage=storage, rho=rho, u=u)
    w = d.weights[:, None, None]
    for steps in (1, 6, 9):
        g.run(steps)
        o.run(steps)
        pg, po = populations_both(d, g, o)
        assert np.max(np.abs(pg - po) / w) <= tol_pop, steps


def test_full_size_throughput_channel_one_step_and_mass():
    """2048 x 512 FP32 D2V37 with the seeded density field: one step against the
    oracle over the whole grid, then 1000 steps conserve mass to FP32 rounding."""
    c = wl.THROUGHPUT_D2V37
    rho = wl.density_field(c["ny"], c["nx"], seed=c["seed"], amp=c["amp"])
    d, g, o = make_pair(c["dvm"], c["N"], c["nx"], c["ny"], kn=c["kn"], ma=c["ma"],
                        storage=c["storage"], rho=rho)
    m0 = g.observe()["mass"]
    g.run(1)
    o.run(1, nthreads=min(16, os.cpu_count() or 1))
    pg, po = populations_both(d, g, o)
    w = d.weights[:, None, None]
    assert np.max(np.abs(pg - po) / w) <= 1e-6
    og, oo = g.observe(), o.observe()
    assert abs(og["mdot"] - oo["mdot"]) <= 1e-5 * abs(oo["mdot"])
    g.run(c["steps"] - 1)
    m1 = g.observe()["mass"]
    assert abs(m1 - m0) <= 1e-7 * m0


def test_bitwise_determinism_and_checkpoint_resume():
    nx, ny = 96, 17
    rho, u = wl.random_state(nx * ny, 2, seed=3, amp=1e-2)
    for storage in ("f64", "f32", "f16dev"):
        d, a, _ = make_pair("D2V37", 4, nx, ny, storage=storage, rho=rho, u=u)
        _, b, _ = make_pair("D2V37", 4, nx, ny, storage=storage, rho=rho, u=u)
        a.run(50)
        b.run(25)
        ck = b.export().clone()
        b.import_(ck)
        b.run(25)
        assert torch.equal(a.export(), b.export()), storage


def test_run_to_tol_matches_oracle_steady_state():
    d, g, o = make_pair("D2V17", 3, 1, 16, kn=0.3)
    r = g.run_to_tol(tol=1e-10, check_every=100, max_steps=200000)
    assert r["converged"]
    o.run(r["steps"])
    assert abs(r["mdot"] - o.observe()["mdot"]) <= 1e-12 * abs(r["mdot"])


def test_f64_scattering_stencil_channel_run():
    """Plane Poiseuille flow on the scattering stencil D2V32 (halo 12), Nx = 1,
    Ny = 36, Kn = 0.2, 3000 steps: mass flow and profile against the oracle."""
    d, g, o = make_pair("D2V32", 4, 1, 36, kn=0.2, ma=1e-3)
    g.run(3000)
    o.run(3000)
    og, oo = g.observe(), o.observe()
    assert _rel(og["u"][..., 0].cpu().numpy(), oo["u"][..., 0]) <= 1e-12
    assert abs(og["mdot"] - oo["mdot"]) <= 1e-12 * abs(oo["mdot"])


def test_slip_and_knudsen_layer_of_gpu_profile():
    """Slip velocity and Knudsen-layer split (lbm_profile_analysis) of a GPU
    channel profile against the oracle's analysis of the oracle's profile."""
    from oracle import profile
    from paper_1510_08886_amd import lbm
    d, g, o = make_pair("D2V37", 4, 1, 40, kn=0.2, ma=1e-3)
    g.run(4000)
    o.run(4000)
    ug = g.observe()["u"][..., 0].mean(dim=-1).cpu().numpy()
    uo = o.observe()["u"][..., 0].mean(axis=-1)
    rg, ro = lbm.profile_analysis(ug), profile.analyse(uo)
    assert abs(rg["slip"] - ro["slip"]) <= 1e-12 * abs(ro["slip"])
    assert np.max(np.abs(rg["u_neq"] - ro["u_neq"])) <= 1e-12 * np.max(np.abs(uo))


@pytest.mark.parametrize("storage,tol_pop", [("f64", 1e-14), ("f32", 1e-7)])
def test_hermite_order_five(storage, tol_pop):
    """Hermite order N = 5 (allowed by the quadrature order 9 of D2V37): a
    random state after 6 steps, element by element against the oracle."""
    nx, ny = 70, 14
    rho, u = wl.random_state(nx * ny, 2, seed=55, amp=3e-2)
    d, g, o = make_pair("D2V37", 5, nx, ny, kn=0.07, ma=3e-2, storage=storage, rho=rho, u=u)
    g.run(6)
    o.run(6)
    pg, po = populations_both(d, g, o)
    # FP64: absolute, as in the other FP64 cases (the order-5 term changes the
    # populations by 2.5e-8 of w here, so dropping it fails); FP32: relative to w
    err = np.abs(pg - po) if storage == "f64" else np.abs(pg - po) / d.weights[:, None, None]
    assert np.max(err) <= tol_pop
    og, oo = g.observe(), o.observe()
    assert abs(og["mdot"] - oo["mdot"]) <= (1e-12 if storage == "f64" else 1e-5) * abs(oo["mdot"])


def test_full_size_scattering_channel_one_step():
    """The D2V32 channel at its benchmark size, 2048 x 512 FP32 (in place, halo
    12, per-XCD tile bands), with the seeded density field: one step against
    the oracle over the whole grid, then the second (gather/scatter) kind."""
    c = wl.SCATTER_D2V32
    rho = wl.density_field(c["ny"], c["nx"])
    d, g, o = make_pair(c["dvm"], c["N"], c["nx"], c["ny"], kn=c["kn"], ma=c["ma"],
                        storage="f32", rho=rho)
    w = d.weights[:, None, None]
    for _ in range(2):
        g.run(1)
        o.run(1, nthreads=min(16, os.cpu_count() or 1))
        pg, po = populations_both(d, g, o)
        assert np.max(np.abs(pg - po) / w) <= 1e-6
    assert abs(g.observe()["mdot"] - o.observe()["mdot"]) <= 1e-5 * abs(o.observe()["mdot"])


def test_full_size_channel_fp16_two_steps():
    """The 2048 x 512 D2V37 channel in FP16-deviation storage (buffer-addressed
    row-grid kernels, hardware stochastic rounding, both in-place kinds): two
    steps against the oracle over the whole grid, to the FP16 bar."""
    c = wl.THROUGHPUT_D2V37
    rho = wl.density_field(c["ny"], c["nx"], seed=c["seed"], amp=c["amp"])
    d, g, o = make_pair(c["dvm"], c["N"], c["nx"], c["ny"], kn=c["kn"], ma=c["ma"],
                        storage="f16dev", rho=rho)
    w = d.weights[:, None, None]
    for _ in range(2):
        g.run(1)
        o.run(1, nthreads=min(16, os.cpu_count() or 1))
        pg, po = populations_both(d, g, o)
        assert np.max(np.abs(pg - po) / w) <= 1e-5
    assert abs(g.observe()["mdot"] - o.observe()["mdot"]) <= 1e-3 * abs(o.observe()["mdot"])


@pytest.mark.parametrize("name,N,nx,ny", [
    ("D2V16", 4, 70, 13),    # no rest velocity, halo 4: two x-tiles plus a ragged tail
    ("D2V16", 3, 3, 9),      # nx < |e_x| = 4: repeated periodic wraps
    ("D2V16", 4, 128, 7),    # aligned rows, ny < 2 * halo: every row a wall row
    ("D2V33", 5, 70, 13),    # quadrature order 9 with the order-5 equilibrium
    ("D2V33", 4, 64, 4),     # ny = largest |e_y| = 4, aligned rows
    ("D2V33", 3, 1, 21),     # streamwise-invariant column
])
@pytest.mark.parametrize("layout", ["in_place", "ping_pong"])
def test_minimal_sets_s5_s6_elementwise(name, N, nx, ny, layout):
    """The minimal models of sets S5 (D2V16) and S6 (D2V33), built on both
    sides from their printed tables (tab:dvmSet5Amin, tab:dvmSet6Amin): a random
    state stepped in place and ping-pong, element by element against the
    oracle (FP64 to 1e-14)."""
    rho, u = wl.random_state(nx * ny, 2, seed=nx * 17 + ny, amp=2e-2)
    d, g, o = make_pair(name, N, nx, ny, kn=0.07, ma=2e-2, rho=rho, u=u, layout=layout)
    for steps in (1, 4):
        g.run(steps)
        o.run(steps)
        pg, po = populations_both(d, g, o)
        assert np.max(np.abs(pg - po)) <= 1e-14, steps
    og, oo = g.observe(), o.observe()
    np.testing.assert_allclose(og["rho"].cpu().numpy(), oo["rho"], rtol=1e-14)
    assert abs(og["mdot"] - oo["mdot"]) <= 1e-12 * abs(oo["mdot"])


@pytest.mark.parametrize("name,N,nx,ny", [
    ("D2V37", 4, 70, 13),    # unaligned rows: 256 consecutive nodes per block, ragged tail
    ("D2V37", 4, 128, 20),   # aligned rows: (x tile, row) grid, per-XCD row bands
    ("D2V37", 3, 192, 11),   # aligned, three 64-node tiles per row
    ("D2V17", 3, 2, 5),      # nx < |e_x|
    ("D2V32", 4, 128, 30),   # halo 12: buffer-addressed row grid
    ("D2V32", 3, 5, 29),     # halo 12, nx < |e_x|
])
@pytest.mark.parametrize("storage,tol", [("f64", 1e-14), ("f32", 1e-8), ("f16dev", 1e-4)])
def test_ping_pong_2d_elementwise(name, N, nx, ny, storage, tol):
    """The 2D ping-pong step (two copies, each step pulls from one into the
    other), which the library takes by default above 512 MiB per copy, forced
    at small sizes: element by element against the oracle after odd and even
    step counts (FP64 absolute; FP32 and FP16 deviations relative to w)."""
    rho, u = wl.random_state(nx * ny, 2, seed=nx * 7 + ny, amp=1e-3)
    d, g, o = make_pair(name, N, nx, ny, kn=0.05, storage=storage, rho=rho, u=u,
                        layout="ping_pong")
    w = d.weights[:, None, None]
    for steps in (1, 6, 9):
        g.run(steps)
        o.run(steps)
        pg, po = populations_both(d, g, o)
        err = np.abs(pg - po) if storage == "f64" else np.abs(pg - po) / w
        assert np.max(err) <= tol, steps
    og, oo = g.observe(), o.observe()
    bar = {"f64": 1e-12, "f32": 1e-5, "f16dev": 1e-3}[storage]
    assert abs(og["mdot"] - oo["mdot"]) <= bar * abs(oo["mdot"])


def test_ping_pong_and_in_place_agree_bitwise():
    """Both layouts perform the same arithmetic per node: a random D2V37 state
    stepped 25 times in place and ping-pong gives identical populations, for
    FP64, FP32 and FP16 deviations (whose stochastic rounding keys on node and
    step, not on the layout)."""
    nx, ny = 128, 24
    rho, u = wl.random_state(nx * ny, 2, seed=44, amp=1e-2)
    for storage in ("f64", "f32", "f16dev"):
        _, a, _ = make_pair("D2V37", 4, nx, ny, storage=storage, rho=rho, u=u, layout="in_place")
        _, b, _ = make_pair("D2V37", 4, nx, ny, storage=storage, rho=rho, u=u, layout="ping_pong")
        a.run(25)
        b.run(25)
        assert torch.equal(a.export(), b.export()), storage


def _full_size_ping_pong(nx, ny, storage, steps, tol, seed):
    from paper_1510_08886_amd import lbm
    d0 = lbm.Dvm.named("D2V37")
    copy = 37 * nx * ny * {"f64": 8, "f32": 4, "f16dev": 2}[storage]
    pop, _ = lbm.state_bytes(d0, lbm.Problem(dim=2, nx=nx, ny=ny, kn=0.05, hermite_order=4,
                                              storage=storage))
    # above 512 MiB per copy: two copies (ping-pong); above 1 GiB for the pair:
    # streaming stores
    assert copy > 512 << 20 and pop == 2 * copy and pop > 1 << 30
    rho = wl.density_field(ny, nx, seed=seed, amp=1e-3)
    d, g, o = make_pair("D2V37", 4, nx, ny, kn=0.05, ma=1e-3, storage=storage, rho=rho)
    w = d.weights[:, None, None]
    for _ in range(steps):
        g.run(1)
        o.run(1, nthreads=min(16, os.cpu_count() or 1))
        pg, po = populations_both(d, g, o)
        err = np.abs(pg - po) if storage == "f64" else np.abs(pg - po) / w
        assert np.max(err) <= tol
        del pg, po
    og, oo = g.observe(), o.observe()
    bar = {"f64": 1e-12, "f32": 1e-5, "f16dev": 1e-3}[storage]
    assert abs(og["mdot"] - oo["mdot"]) <= bar * abs(oo["mdot"])
    mass_bar = {"f64": 1e-12, "f32": 1e-8, "f16dev": 1e-6}[storage]
    assert abs(og["mass"] - oo["mass"]) <= mass_bar * oo["mass"]


def test_full_size_ping_pong_f64_2048x1024():
    """D2V37 FP64 2048 x 1024: 620 MB per copy, so the default layout is two
    copies stepped ping-pong with streaming stores. Two steps over the whole
    grid against the oracle to 1e-14."""
    _full_size_ping_pong(2048, 1024, "f64", 2, 1e-14, seed=1024)


def test_full_size_ping_pong_f32_4096x1024():
    """D2V37 FP32 4096 x 1024 (620 MB per copy, 1.24 GB for the pair): the
    default ping-pong step with streaming stores, one step over the whole grid
    against the oracle to 1e-6 of w."""
    _full_size_ping_pong(4096, 1024, "f32", 1, 1e-6, seed=4096)


def test_full_size_ping_pong_f16dev_4096x2048():
    """D2V37 FP16 deviations 4096 x 2048 (620 MB per copy): the buffer-addressed
    ping-pong step with streaming stores and stochastic rounding, one step over
    the whole grid against the oracle to 1e-5 of w."""
    _full_size_ping_pong(4096, 2048, "f16dev", 1, 1e-5, seed=2048)


@pytest.mark.parametrize("name,N,nx,ny,band_rows", [
    ("D2V37", 4, 128, 20, 0),    # aligned rows, default bands
    ("D2V37", 4, 70, 13, 0),     # partial second strip (6 columns), unaligned
    ("D2V37", 4, 130, 24, 5),    # bands of 5 rows: halos reach across several bands
    ("D2V37", 3, 64, 64, 1),     # one-row bands
    ("D2V17", 3, 2, 5, 0),       # nx < |e_x|: the widened tile repeats columns
    ("D2V17", 3, 1, 21, 2),      # streamwise-invariant column, two-row bands
    ("D2V37", 5, 192, 11, 3),    # Hermite order 5; every band touches a wall
    ("D2V33", 5, 96, 17, 7),     # halo 4
    ("D2V16", 4, 64, 9, 0),      # halo 4, no rest velocity, ny < 2 * halo
])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16dev", "f32raw"])
@pytest.mark.parametrize("mode", [1, 2, 3])
def test_pair_steps_equal_single_steps(name, N, nx, ny, band_rows, storage, mode):
    """Two steps per launch (the intermediate state in an LDS ring; mode 1:
    all waves alternate between the two steps, mode 2: producer and consumer
    waves, mode 3: two producer groups on alternate chunks and consumer waves)
    against one launch per step:
    bit-identical populations after even and odd step counts (an odd count
    ends with one single step), on random states, for every storage; FP64 also
    element by element against the oracle."""
    from paper_1510_08886_amd import lbm
    rho, u = wl.random_state(nx * ny, 2, seed=nx * 3 + ny, amp=1e-2)
    d, a, o = make_pair(name, N, nx, ny, kn=0.07, ma=2e-2, storage=storage, rho=rho, u=u,
                        layout="ping_pong")
    _, b, _ = make_pair(name, N, nx, ny, kn=0.07, ma=2e-2, storage=storage, rho=rho, u=u,
                        layout="ping_pong")
    b.set_graph_steps(0).set_pair_steps(False)
    try:
        a.set_graph_steps(0).set_pair_steps(mode, band_rows)
        a.run(2)
    except lbm.LbmError as err:
        assert mode in (2, 3) and err.code == lbm.LBM_E_UNSUPPORTED
        pytest.skip("the producer/consumer ring of this set and storage does not fit the LDS")
    b.run(2)
    if storage == "f64":
        o.run(2)
    for steps in (0, 7, 4):
        a.run(steps)
        b.run(steps)
        assert torch.equal(a.export(), b.export()), steps
        if storage == "f64":
            o.run(steps)
            pg, po = populations_both(d, a, o)
            assert np.max(np.abs(pg - po)) <= 1e-14, steps
    ma, mb = a.observe(), b.observe()
    assert ma["mdot"] == mb["mdot"] and ma["mass"] == mb["mass"]


def test_pair_steps_mode_validation():
    """Modes 0-3 are accepted for a 2D ping-pong problem (the twin-producer
    mode 3 is compiled for every set that has the two-step kernel); anything
    else is LBM_E_INVALID, and in-place stepping refuses two-step launches."""
    from paper_1510_08886_amd import lbm
    d, a, _ = make_pair("D2V37", 4, 64, 9, storage="f32", layout="ping_pong")
    for mode in (0, 1, 2, 3):
        a.set_pair_steps(mode)
    for mode in (4, -1):
        with pytest.raises(lbm.LbmError) as e:
            a.set_pair_steps(mode)
        assert e.value.code == lbm.LBM_E_INVALID
    _, b, _ = make_pair("D2V37", 4, 64, 9, storage="f32", layout="in_place")
    with pytest.raises(lbm.LbmError) as e:
        b.set_pair_steps(3)
    assert e.value.code == lbm.LBM_E_UNSUPPORTED


@pytest.mark.parametrize("mode", [1, 3])
def test_pair_steps_full_size_channel(mode):
    """The 2048 x 512 D2V37 FP32 throughput channel stepped ping-pong with two
    steps per launch (default bands; mode 3 is how the library steps this
    channel by default): 10 steps bit-identical to single-step launches, then
    two more against the oracle over the grid."""
    c = wl.THROUGHPUT_D2V37
    rho = wl.density_field(c["ny"], c["nx"], seed=c["seed"], amp=c["amp"])
    d, a, o = make_pair(c["dvm"], c["N"], c["nx"], c["ny"], kn=c["kn"], ma=c["ma"],
                        storage="f32", rho=rho, layout="ping_pong")
    _, b, _ = make_pair(c["dvm"], c["N"], c["nx"], c["ny"], kn=c["kn"], ma=c["ma"],
                        storage="f32", rho=rho, layout="ping_pong")
    a.set_pair_steps(mode)
    b.set_pair_steps(False)
    a.run(10)
    b.run(10)
    assert torch.equal(a.export(), b.export())
    o.run(10, nthreads=min(16, os.cpu_count() or 1))
    a.run(2)
    o.run(2, nthreads=min(16, os.cpu_count() or 1))
    pg, po = populations_both(d, a, o)
    assert np.max(np.abs(pg - po) / d.weights[:, None, None]) <= 1e-6


@pytest.mark.parametrize("name,N,nx,ny", [
    ("D2V37", 4, 70, 13),    # unaligned rows, ragged tail
    ("D2V37", 4, 128, 20),   # aligned rows, both in-place kinds on the row grid
    ("D2V17", 3, 2, 5),      # nx < |e_x|: mirrored sources wrap in x
    ("D2V33", 5, 64, 9),     # halo 4, order-5 equilibrium
    ("D2V32", 4, 128, 30),   # halo 12, buffer-addressed row grid
    ("D2V32", 3, 5, 29),     # halo 12, nx < |e_x|
    ("D2V37", 4, 1, 21),     # one column: in place this is the one-workgroup resident kernel
])
@pytest.mark.parametrize("layout", ["auto", "ping_pong"])
@pytest.mark.parametrize("alpha", [0.0, 0.3, 0.75])
def test_accommodation_elementwise(name, N, nx, ny, layout, alpha):
    """Maxwell walls with a diffuse fraction alpha and the rest reflected
    specularly, FP64 (such problems step ping-pong: the specular partner is
    another node's leaving population, which the in-place kernels overwrite in
    the same step), element by element against the oracle, then the observed
    moments (which read the specular partners too)."""
    rho, u = wl.random_state(nx * ny, 2, seed=nx * 5 + ny, amp=2e-2)
    d, g, o = make_pair(name, N, nx, ny, kn=0.07, ma=2e-2, rho=rho, u=u, layout=layout,
                        alpha=alpha)
    for steps in (1, 6, 9):
        g.run(steps)
        o.run(steps)
        pg, po = populations_both(d, g, o)
        assert np.max(np.abs(pg - po)) <= 1e-14, steps
    og, oo = g.observe(), o.observe()
    np.testing.assert_allclose(og["rho"].cpu().numpy(), oo["rho"], rtol=1e-14)
    np.testing.assert_allclose(og["u"].cpu().numpy()[..., :2], oo["u"][..., :2], rtol=0, atol=1e-15)


@pytest.mark.parametrize("storage,tol_pop", [("f32", 1e-8), ("f16dev", 1e-4)])
def test_accommodation_low_precision(storage, tol_pop):
    nx, ny = 128, 24
    rho, u = wl.random_state(nx * ny, 2, seed=61, amp=1e-3)
    d, g, o = make_pair("D2V37", 4, nx, ny, kn=0.05, storage=storage, rho=rho, u=u,
                        alpha=0.6)
    w = d.weights[:, None, None]
    for steps in (1, 40, 59):
        g.run(steps)
        o.run(steps)
        pg, po = populations_both(d, g, o)
        assert np.max(np.abs(pg - po) / w) <= tol_pop, steps


@pytest.mark.parametrize("mode", [1, 2, 3])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_accommodation_pair_steps(mode, storage):
    """Two steps per launch with specular partners taken from the LDS ring
    (second step) and from HBM (first step): bitwise equal to single steps."""
    nx, ny = 130, 24
    rho, u = wl.random_state(nx * ny, 2, seed=62, amp=1e-2)
    _, a, _ = make_pair("D2V37", 4, nx, ny, storage=storage, rho=rho, u=u, layout="ping_pong",
                        alpha=0.45)
    _, b, _ = make_pair("D2V37", 4, nx, ny, storage=storage, rho=rho, u=u, layout="ping_pong",
                        alpha=0.45)
    a.set_graph_steps(0).set_pair_steps(mode, 5)
    b.set_graph_steps(0).set_pair_steps(False)
    for steps in (2, 7, 4):
        a.run(steps)
        b.run(steps)
        assert torch.equal(a.export(), b.export()), steps


def test_specular_channel_accelerates_freely():
    """alpha = 0 from rest (D2V37 FP64, 64 x 7): u_x = (n + 1/2) g dt at every
    node after n steps, u_y = 0 (the plug flow of fully specular walls)."""
    d, g, _ = make_pair("D2V37", 4, 64, 7, kn=0.2, alpha=0.0)
    par = g.params
    g.run(33)
    o = g.observe()
    ux = o["u"][..., 0].cpu().numpy()
    want = 33.5 * par.g[0] * par.dt
    assert np.max(np.abs(ux - want)) <= 1e-12 * want
    assert np.max(np.abs(o["u"][..., 1].cpu().numpy())) <= 1e-16


def _throughput_golden():
    from pathlib import Path
    rows = [l.split() for l in (Path(__file__).resolve().parent / "golden" / "throughput_d2v37.txt")
            .read_text().splitlines() if l and not l.startswith("#")]
    g = {"mdot": {}, "uxrow": {}, "col": {}}
    for r in rows:
        if r[0] == "mdot":
            g["mdot"][int(r[1])] = (float(r[2]), float(r[3]))
        elif r[0] == "uxrow":
            g["uxrow"][int(r[1])] = float(r[2])
        elif r[0] == "col":
            g["col"][(int(r[1]), int(r[2]))] = tuple(float(x) for x in r[3:6])
        elif r[0] == "steps":
            g["steps"] = int(r[1])
    return g


@pytest.mark.parametrize("layout,pair", [("auto", 0), ("ping_pong", 2), ("ping_pong", 3)])
def test_throughput_channel_1000_steps_against_oracle(layout, pair):
    """The 2048 x 512 D2V37 FP32 throughput channel, 1000 steps from the seeded
    density, against the stored FP64 oracle run (tests/golden/throughput_d2v37.txt):
    the mass flow every 100 steps and the row-averaged u_x within 1e-5
    relative, rho on four sampled columns within 1e-5 elementwise, and u_x,
    u_y there within 1e-5 of the column's largest |u_x| (FP32 deviation
    storage errs on the velocity by an absolute amount on the scale of the
    flow, so u_y, a thousand times smaller than u_x here, is held to the flow's
    scale, not its own). Default in-place stepping, and ping-pong with two
    steps per launch."""
    c = wl.THROUGHPUT_D2V37
    g = _throughput_golden()
    rho = wl.density_field(c["ny"], c["nx"], seed=c["seed"], amp=c["amp"])
    from paper_1510_08886_amd import lbm
    d = lbm.Dvm.named(c["dvm"])
    prob = lbm.Problem(dim=2, nx=c["nx"], ny=c["ny"], kn=c["kn"], ma=c["ma"], hermite_order=c["N"],
                       storage="f32", layout=layout)
    s = lbm.Solver(d, prob)
    s.init(torch.from_numpy(rho))
    if pair:
        s.set_pair_steps(pair)
    done = 0
    for step in sorted(g["mdot"]):
        s.run(step - done)
        done = step
        ob = s.observe()
        want_md, want_mass = g["mdot"][step]
        assert abs(ob["mdot"] - want_md) <= 1e-5 * abs(want_md), step
        assert abs(ob["mass"] - want_mass) <= 1e-9 * want_mass, step
    assert done == g["steps"] == c["steps"]
    u = ob["u"].cpu().numpy()
    r = ob["rho"].cpu().numpy()
    ux_row = u[..., 0].mean(axis=1)
    want_row = np.array([g["uxrow"][j] for j in range(c["ny"])])
    assert np.max(np.abs(ux_row - want_row)) <= 1e-5 * np.max(np.abs(want_row))
    cols = sorted({i for i, _ in g["col"]})
    for i in cols:
        ref = np.array([g["col"][(i, j)] for j in range(c["ny"])])
        np.testing.assert_allclose(r[:, i], ref[:, 0], rtol=1e-5, atol=0)
        scale = np.max(np.abs(ref[:, 1]))
        for k in (1, 2):
            assert np.max(np.abs(u[:, i, k - 1] - ref[:, k])) <= 1e-5 * scale, (i, k)
    s.close()


@pytest.mark.parametrize("name,N,nx,ny,layout", [
    ("D2V17", 3, 1, 40, "auto"),        # one column: resident stepping
    ("D2V37", 4, 70, 13, "auto"),       # in place, ragged tiles
    ("D2V37", 4, 128, 20, "ping_pong"), # aligned rows, ping-pong
    ("D2V37", 5, 64, 9, "auto"),        # Hermite order 5
])
def test_f32sr_storage(name, N, nx, ny, layout):
    """FP32 deviations collided in FP64 with stochastic rounding: element by
    element against the oracle (each step's rounding is at most one FP32 ulp
    of the deviation, unbiased), deterministic (two runs bit for bit), and the
    mass flow within 1e-7 after 300 steps."""
    rho, u = wl.random_state(nx * ny, 2, seed=5 * nx + ny, amp=1e-3)
    d, g, o = make_pair(name, N, nx, ny, kn=0.05, storage="f32sr", rho=rho, u=u, layout=layout)
    _, h, _ = make_pair(name, N, nx, ny, kn=0.05, storage="f32sr", rho=rho, u=u, layout=layout)
    w = d.weights[:, None, None]
    for steps in (1, 22, 277):
        g.run(steps)
        h.run(steps)
        o.run(steps)
        pg, po = populations_both(d, g, o)
        assert np.max(np.abs(pg - po) / w) <= 1e-8, steps
        assert torch.equal(g.export(), h.export()), steps
    og, oo = g.observe(), o.observe()
    assert abs(og["mdot"] - oo["mdot"]) <= 1e-7 * abs(oo["mdot"])


def test_f32sr_is_unsupported_outside_the_channel_sets():
    from paper_1510_08886_amd import lbm
    for name, dim, nz in (("D2V32", 2, 1), ("D3V39", 3, 8)):
        d = lbm.Dvm.named(name)
        prob = lbm.Problem(dim=dim, nx=8, ny=16, nz=nz, kn=0.1, hermite_order=3, storage="f32sr")
        with pytest.raises(lbm.LbmError) as e:
            lbm.Solver(d, prob)
        assert e.value.code == lbm.LBM_E_UNSUPPORTED
