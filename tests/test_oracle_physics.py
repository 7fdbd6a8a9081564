"""Pins of the oracle time stepper against what the paper and the mathematics fix.

* equilibrium moment identities (Section III, case 1 of the low-Ma error
  estimate, Eq. ce.34 and Appendix C): for k <= N and k + N <= Q the discrete
  moments of f^(0) equal the Maxwellian's exactly;
* force moments (Eq. nm.4 with the orthogonality Eq. orth): sum F = 0,
  sum F xi = rho g (used in Eq. nm.10), sum F xi xi = rho (g u + u g), and the
  third moment of the continuous force term -g.grad_xi f, g_i Pi_jk + perms;
* collision leaves f^(0) unchanged when g = 0, and a uniform rest state is a
  fixed point of a full step including the walls (Psi = 1 for uniform density,
  Section IV.A and Section V);
* exact mass conservation, per-element balance of absorbed and emitted mass at
  the walls (Eq. nm.15, discrete reading), momentum injection rho g dt per node
  and step (Eq. nm.8 with omega (tau + dt/2) = dt);
* mirror symmetry of the channel and exact reversal under g -> -g;
* the Navier-Stokes limit of plane Poiseuille flow: curvature -g/nu in the bulk
  and m * 6 Kn -> 1 (Eq. pf.2) as Kn -> 0 with a roughly constant first-order
  slip offset (the offset itself is not printed in the paper: parity unpinned);
* a pure-Python dictionary implementation agrees with the C oracle on tiny grids.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import dvm, stepper
from tests import bruteforce
from tests.golden.tables import load_dvm_tables

# the channel / duct models, and the scattering stencils D2V32 (set S7) and
# D3V96 (set S4) built from their printed tables
CASES = [("D2V17", 3), ("D2V37", 4), ("D3V39", 3), ("D2V32", 4), ("D3V96", 3)]
TABLE_MODELS = ("D2V32", "D3V96")


def _dvm(name):
    if name in TABLE_MODELS:
        m = {t["label"]: t for t in load_dvm_tables()}[name]
        return dvm.make_dvm(m["D"], m["gens"], m["weights"], m["c"], m["Q"])
    return dvm.named_dvm(name)


def _kw(name, nx, ny, nz=1):
    """Grid arguments with walls on y (and z in 3D), at least as wide as the
    largest wall-normal velocity component."""
    d = _dvm(name)
    hn = int(np.abs(d.velocities[:, 1:]).max())
    kw = dict(nx=nx, ny=max(ny, hn + 1))
    if d.dim == 3:
        kw.update(nz=max(nz, hn + 1), walls_z=True)
    return kw


def _maxwell_moment(rho, u, exps):
    """Moment of rho * N(u, I): prod_d E[(u_d + Z)^a_d]."""
    out = rho
    for ud, a in zip(u, exps):
        s = 0.0
        for k in range(0, a + 1, 2):
            s += math.comb(a, k) * ud ** (a - k) * (math.prod(range(k - 1, 0, -2)) if k else 1)
        out *= s
    return out


def _solver(name, N, **kw):
    d = _dvm(name)
    hn = int(np.abs(d.velocities[:, 1:]).max())
    defaults = dict(nx=1, ny=max(8, hn + 1), nz=(max(8, hn + 1) if d.dim == 3 else 1), kn=0.1,
                    ma=1e-3, N=N)
    defaults.update(kw)
    return stepper.OracleSolver(d, **defaults)


@pytest.mark.parametrize("name,N", CASES)
def test_equilibrium_moment_identities(oracle_lib, name, N):
    s = _solver(name, N)
    d = s.dvm
    rng = np.random.default_rng(11)
    for _ in range(3):
        rho = 1.0 + 0.2 * rng.random()
        u = 0.15 * rng.normal(size=d.dim)
        feq = s.equilibrium(rho, u)
        xi = d.xi
        for k in range(0, N + 1):
            if k + N > d.Q:
                continue
            for exps in itertools.product(range(k + 1), repeat=d.dim):
                if sum(exps) != k:
                    continue
                got = float(np.sum(feq * np.prod(xi ** np.array(exps), axis=1)))
                want = _maxwell_moment(rho, u, exps)
                assert abs(got - want) < 2e-14 * max(1.0, abs(want))
        # order N+1 is not captured by the truncated expansion
        big = int(np.argmax(np.abs(u)))
        exps = tuple(N + 1 if dd == big else 0 for dd in range(d.dim))
        got = float(np.sum(feq * xi[:, big] ** (N + 1)))
        assert abs(got - _maxwell_moment(rho, u, exps)) > 1e-8


@pytest.mark.parametrize("name,N", CASES)
def test_tensor_equilibrium_matches_scalar_recurrence(oracle_lib, name, N):
    s = _solver(name, N)
    d = s.dvm
    rng = np.random.default_rng(3)
    rho = 1.07
    u = 0.05 * rng.normal(size=d.dim)
    feq = s.equilibrium(rho, u)
    ref = [bruteforce.equilibrium(d.weights[a], d.xi[a], rho, u, N) for a in range(d.V)]
    np.testing.assert_allclose(feq, ref, rtol=0, atol=2e-16)


@pytest.mark.parametrize("name,N", CASES)
def test_force_moments(oracle_lib, name, N):
    s = _solver(name, N)
    d = s.dvm
    g = np.array(s.params.g[: d.dim]) * 50.0 + np.array([0.0, 0.01, 0.02][: d.dim])
    s._p.g[0], s._p.g[1], s._p.g[2] = (list(g) + [0.0])[:3]
    rng = np.random.default_rng(5)
    rho = 0.93
    u = 0.05 * rng.normal(size=d.dim)
    A = rng.normal(size=(d.dim, d.dim))
    Pi = rho * np.eye(d.dim) + 0.1 * (A + A.T)
    F = s.force(rho, u, Pi)
    xi = d.xi
    assert abs(F.sum()) < 1e-16
    np.testing.assert_allclose(xi.T @ F, rho * g, rtol=0, atol=1e-16)
    M2 = np.einsum("a,ai,aj->ij", F, xi, xi)
    np.testing.assert_allclose(M2, rho * (np.outer(g, u) + np.outer(u, g)), rtol=0, atol=1e-16)
    M3 = np.einsum("a,ai,aj,ak->ijk", F, xi, xi, xi)
    want = (np.einsum("i,jk->ijk", g, Pi) + np.einsum("j,ik->ijk", g, Pi)
            + np.einsum("k,ij->ijk", g, Pi))
    np.testing.assert_allclose(M3, want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("name,N", CASES)
def test_collision_fixed_point_without_force(oracle_lib, name, N):
    s = _solver(name, N, g=(0.0, 0.0, 0.0))
    rng = np.random.default_rng(9)
    for _ in range(3):
        rho = 1.0 + 0.1 * rng.random()
        u = 0.01 * rng.normal(size=s.dvm.dim)
        f0 = s.equilibrium(rho, u)
        out = s.collide_node(f0)
        np.testing.assert_allclose(out, f0, rtol=0, atol=2e-16)


@pytest.mark.parametrize("name,N", CASES)
def test_uniform_rest_state_is_fixed_point_with_walls(oracle_lib, name, N):
    kw = dict(_kw(name, 3, 7, 6), g=(0.0, 0.0, 0.0))
    s = _solver(name, N, **kw)
    s.init(rho=np.full(s.nodes, 1.3))
    f0 = s.f.copy()
    s.run(3)
    # rho_eff = A / D with A and D FP64 sums of up to ~300 crossing populations
    # (12 wall rows for D2V32, 7 rows on four faces for D3V96): rounding of
    # up to a few 1e-14 relative; a wrong wall rule gives O(1) errors
    np.testing.assert_allclose(s.f, f0, rtol=5e-14, atol=0)


def _random_state(s, seed, amp=1e-3):
    rng = np.random.default_rng(seed)
    rho = 1.0 + amp * rng.standard_normal(s.nodes)
    u = np.zeros((s.nodes, 3))
    u[:, : s.dim] = amp * rng.standard_normal((s.nodes, s.dim))
    return s.init(rho=rho, u=u)


@pytest.mark.parametrize("name,N", CASES)
def test_mass_conservation(oracle_lib, name, N):
    s = _random_state(_solver(name, N, **_kw(name, 4, 9, 7)), 1)
    m0 = s.f.sum()
    s.run(300)
    # rounding only: a random walk of ~1e-16 per step
    assert abs(s.f.sum() - m0) / m0 < 5e-14


def test_mass_conservation_config1_long(oracle_lib):
    s = _random_state(_solver("D2V17", 3, nx=1, ny=40), 2)
    m0 = s.f.sum()
    s.run(20000)
    assert abs(s.f.sum() - m0) / m0 < 1e-13


@pytest.mark.parametrize("name,N", CASES)
def test_wall_balance_per_element(oracle_lib, name, N):
    """Absorbed mass per element equals emitted mass per element, checked by an
    independent enumeration of the stream output."""
    s = _random_state(_solver(name, N, **_kw(name, 5, 7, 6)), 4, amp=1e-2)
    s.run(2)
    A, Dn = s.wall_balance()
    pre = s.stream()
    d = s.dvm
    nx, ny, nz = s.nx, s.ny, s.nz
    emitted = np.zeros_like(A)
    shape = (nz, ny, nx)
    for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
        n = np.ravel_multi_index((k, j, i), shape)
        for a in range(d.V):
            e = list(d.velocities[a]) + [0] * (3 - d.dim)
            js, ks = j - e[1], k - e[2]
            oy = not (0 <= js < ny)
            oz = s.walls_z and not (0 <= ks < nz)
            if not (oy or oz):
                continue
            assert Dn.sum() > 0
            # first face crossed going outward from the node along -e (ties: y);
            # element = the node's own cell on that face
            if oy and oz:
                ty = ((ny - 0.5 if -e[1] > 0 else -0.5) - j) / -e[1]
                tz = ((nz - 0.5 if -e[2] > 0 else -0.5) - k) / -e[2]
                use_z = tz < ty
            else:
                use_z = oz
            if use_z:
                face = 2 if e[2] > 0 else 3
                el = j * nx + i
            else:
                face = 0 if e[1] > 0 else 1
                el = k * nx + i
            emitted[face, el] += pre[n, a]
    np.testing.assert_allclose(emitted, A, rtol=1e-13, atol=1e-15)
    # every element with absorbed mass also has emitting slots
    assert np.all(Dn[A > 0] > 0)
    # streaming alone conserves mass
    assert abs(pre.sum() - s.f.sum()) < 1e-13 * s.f.sum()


@pytest.mark.parametrize("name,N", CASES)
def test_momentum_injection_per_node(oracle_lib, name, N):
    s = _random_state(_solver(name, N, **_kw(name, 2, 5, 4)), 6, amp=1e-2)
    pre = s.stream()
    post = s.collide(pre)
    rho = pre.sum(axis=1)
    dj = (post - pre) @ s.dvm.xi
    want = rho[:, None] * np.array(s.params.g[: s.dim])[None, :] * s.params.dt
    # (post - pre) . xi cancels O(0.1) populations: rounding ~1e-17 absolute
    np.testing.assert_allclose(dj, want, rtol=0, atol=2e-16)
    # per-node mass: two sums of up to 96 populations, ~1e-15 relative rounding
    np.testing.assert_allclose(post.sum(axis=1), rho, rtol=4e-15)


def test_channel_symmetry_and_force_reversal(oracle_lib):
    s1 = _solver("D2V37", 4, nx=1, ny=12).init().run(400)
    o1 = s1.observe()
    ux = o1["u"][:, 0, 0]
    assert np.max(np.abs(ux - ux[::-1])) < 1e-12 * np.max(np.abs(ux))
    g = s1.params.g
    s2 = _solver("D2V37", 4, nx=1, ny=12, g=(-g[0], 0.0, 0.0)).init().run(400)
    o2 = s2.observe()
    np.testing.assert_allclose(o2["u"][:, 0, 0], -ux, rtol=1e-12, atol=0)


def test_x_invariance_of_uniform_start(oracle_lib):
    a = _solver("D2V17", 3, nx=1, ny=10).init().run(50).observe()
    b = _solver("D2V17", 3, nx=3, ny=10).init().run(50).observe()
    for i in range(3):
        np.testing.assert_allclose(b["u"][:, i, 0], a["u"][:, 0, 0], rtol=1e-14)


@pytest.mark.slow
def test_navier_stokes_limit(oracle_lib):
    """Bulk curvature -g/nu and m * 6 Kn -> 1 with an O(1) slip offset."""
    offsets, ratios = [], []
    for kn in (0.02, 0.01, 0.005):
        s = _solver("D2V17", 3, nx=1, ny=40, kn=kn).init()
        p = s.params
        s.run(int(14 / (math.pi ** 2 * p.tau) / p.dt))
        o = s.observe()
        ux = o["u"][:, 0, 0]
        y = (np.arange(40) + 0.5) / 40 - 0.5
        mid = np.abs(y) < 0.25
        curv = np.polyfit(y[mid], ux[mid], 2)[0]
        # NS: nu u'' = -g  ->  u = const - g y^2 / (2 nu); g / (2 nu) = 4 Ma
        assert abs(curv / (-p.g[0] / (2 * p.tau)) - 1) < 1e-4
        offsets.append(o["mdot"] - 1 / (6 * kn))
        ratios.append(o["mdot"] * 6 * kn)
    assert ratios[0] > ratios[1] > ratios[2] > 1.0
    assert ratios[2] < 1.05
    assert max(offsets) - min(offsets) < 0.15 * np.mean(offsets)


def test_psi_close_to_one_at_steady_state(oracle_lib):
    s = _solver("D2V17", 3, nx=1, ny=20, kn=0.1).init().run(6000)
    A, Dn = s.wall_balance()
    o = s.observe()
    rho_first = o["rho"][0, 0]
    for face in (0, 1):
        psi = A[face, 0] / Dn[face, 0] / rho_first
        assert abs(psi - 1) < 1e-6          # 1 + O(Ma^2), Ma = 1e-3
    uy = o["u"][:, 0, 1]
    assert np.max(np.abs(uy)) < 1e-9


@pytest.mark.parametrize("name,N", [("D2V17", 3), ("D2V37", 4)])
def test_bruteforce_python_matches_c_oracle(oracle_lib, name, N):
    nx, ny = 3, 6
    s = _random_state(_solver(name, N, nx=nx, ny=ny, ma=5e-2), 8, amp=2e-2)
    d = s.dvm
    vels = [tuple(int(v) for v in e) for e in d.velocities]
    f = {}
    for j in range(ny):
        for i in range(nx):
            n = j * nx + i
            for a, e in enumerate(vels):
                f[(i, j, e)] = s.f[n, a]
    p = s.params
    for _ in range(3):
        f = bruteforce.step(f, vels, list(d.weights), d.c, nx, ny, N, p.tau, p.dt, p.g[:2])
    s.run(3)
    for j in range(ny):
        for i in range(nx):
            n = j * nx + i
            for a, e in enumerate(vels):
                assert abs(f[(i, j, e)] - s.f[n, a]) < 1e-15


def test_duct_golden_file_is_consistent():
    """The stored oracle duct run (tests/golden/duct_d3v39_mdot.txt): mass of
    the 256 x 256 column stays rho0 * nodes, and the flow started from rest
    accelerates monotonically over the first 500 steps."""
    from pathlib import Path
    rows = [l.split() for l in (Path(__file__).resolve().parent / "golden" / "duct_d3v39_mdot.txt")
            .read_text().splitlines() if l and not l.startswith("#")]
    steps = [int(r[0]) for r in rows]
    mdot = [float(r[1]) for r in rows]
    mass = [float(r[2]) for r in rows]
    assert steps == list(range(50, 501, 50))
    assert all(abs(m - 65536.0) <= 1e-12 * 65536.0 for m in mass)
    assert all(b > a for a, b in zip(mdot, mdot[1:]))


def test_sweep_golden_file_matches_recipe_and_oracle():
    """The stored oracle mass flows of the sweep's smallest channels
    (tests/golden/sweep_d2v37_mdot.txt) belong to the current sweep recipe, and
    re-running the oracle on the two cheapest reproduces them."""
    from pathlib import Path

    from tests.golden import make_sweep_golden as msg
    rows = [l.split() for l in (Path(__file__).resolve().parent / "golden" / "sweep_d2v37_mdot.txt")
            .read_text().splitlines() if l and not l.startswith("#")]
    assert [(int(r[0]), int(r[1]), float(r[2])) for r in rows] == msg.channels()
    for r in rows[:2]:
        o = stepper.OracleSolver(dvm.named_dvm("D2V37"), nx=1, ny=int(r[1]), kn=float(r[2]),
                                 ma=1e-3, N=4).init()
        o.run(int(r[3]))
        assert abs(o.observe()["mdot"] - float(r[4])) <= 1e-14 * float(r[4])


def test_channel_golden_file_matches_oracle():
    """The stored 20000-step D2V17 channel (tests/golden/channel_d2v17.txt):
    mirror-symmetric profile, mass rho0 * ny, and a re-run of the oracle
    reproduces it."""
    from pathlib import Path
    rows = [l.split() for l in (Path(__file__).resolve().parent / "golden" / "channel_d2v17.txt")
            .read_text().splitlines() if l and not l.startswith("#")]
    kv = {r[0]: float(r[1]) for r in rows if r[0] != "ux"}
    ux = np.array([float(r[2]) for r in rows if r[0] == "ux"])
    assert len(ux) == 40 and kv["steps"] == 20000
    # mirror nodes sum their populations in different orders: rounding at the
    # scale of the populations (~1), not of u (~1e-3)
    assert np.max(np.abs(ux - ux[::-1])) <= 1e-15
    assert abs(kv["mass"] - 40.0) <= 1e-13 * 40.0
    o = stepper.OracleSolver(dvm.named_dvm("D2V17"), nx=1, ny=40, kn=0.1, ma=1e-3, N=3).init()
    o.run(20000)
    ob = o.observe()
    assert abs(ob["mdot"] - kv["mdot"]) <= 1e-14 * kv["mdot"]
    assert np.max(np.abs(ob["u"][:, 0, 0] - ux)) <= 1e-14 * np.max(ux)


def test_converged_golden_files_match_recipes_and_oracle():
    """The stored converged oracle runs (tests/golden/sweep_d2v37_converged.txt,
    serve_sample_converged.txt) belong to the current sweep recipe and serving
    sample; each solve stopped at the first check whose relative change was
    below the tolerance; and re-running the oracle on the cheapest stored solve
    reproduces its first stored value."""
    from tests.golden import make_converged_golden as mcg
    from tests.golden.converged import SERVE, SWEEP, load_converged
    for path, jobs in ((SWEEP, mcg.sweep_jobs()), (SERVE, mcg.serve_sample())):
        if not path.exists():
            pytest.skip(f"{path.name} not generated yet")
        gold = load_converged(path)
        assert sorted(gold) == sorted(j[0] for j in jobs)
        for key, name, ny, kn in jobs:
            g = gold[key]
            assert (g["dvm"], g["ny"], g["kn"]) == (name, ny, kn)
            assert g["stop"] is not None
            steps = sorted(g["mdot"])
            assert steps[0] == mcg.CHECK and steps[-1] == g["stop"] + mcg.WINDOW_AFTER
            assert all(b - a == mcg.CHECK for a, b in zip(steps, steps[1:]))
            m = g["mdot"]
            # the stop is the first stored check meeting the tolerance
            for s in steps[1:]:
                rel = abs(m[s] - m[s - mcg.CHECK]) < mcg.TOL * abs(m[s])
                assert rel == (s >= g["stop"]) or s > g["stop"], (key, s)
            assert abs(m[g["stop"]] - m[g["stop"] - mcg.CHECK]) < mcg.TOL * abs(m[g["stop"]])
        key = min(gold, key=lambda k: gold[k]["ny"] * min(gold[k]["mdot"]))
        g = gold[key]
        s0 = min(g["mdot"])
        o = stepper.OracleSolver(dvm.named_dvm(g["dvm"]), nx=1, ny=g["ny"], kn=g["kn"], ma=1e-3,
                                 N=mcg.N_OF[g["dvm"]]).init()
        o.run(s0)
        assert abs(o.observe()["mdot"] - g["mdot"][s0]) <= 1e-14 * abs(g["mdot"][s0])


def test_throughput_golden_file_matches_recipe():
    """The stored 1000-step oracle run of the 2048 x 512 throughput channel
    (tests/golden/throughput_d2v37.txt): its mass is the seeded density's
    sum at every check (exact conservation), the mass flow grows from rest,
    the row-averaged u_x is near mirror-symmetric (exactly so but for the 1e-3
    random density) and non-slip (u_x > 0 at the wall rows), and the stored
    columns' densities are the seeded ones up to O(Ma) changes."""
    import lbm_workloads as wl
    from tests.test_gpu_parity import _throughput_golden
    c = wl.THROUGHPUT_D2V37
    g = _throughput_golden()
    rho0 = wl.density_field(c["ny"], c["nx"], seed=c["seed"], amp=c["amp"])
    assert g["steps"] == c["steps"] and sorted(g["mdot"]) == list(range(100, 1001, 100))
    for step, (md, mass) in g["mdot"].items():
        assert abs(mass - rho0.sum()) <= 1e-12 * rho0.sum(), step
    mds = [g["mdot"][k][0] for k in sorted(g["mdot"])]
    assert all(b > a > 0 for a, b in zip(mds, mds[1:]))
    ux = np.array([g["uxrow"][j] for j in range(c["ny"])])
    assert np.max(np.abs(ux - ux[::-1])) <= 1e-2 * np.max(ux)
    assert ux[0] > 0 and ux[-1] > 0
    r0 = rho0.reshape(c["ny"], c["nx"])
    for (i, j), (rho, _, _) in g["col"].items():
        assert abs(rho - r0[j, i]) <= 5e-3
