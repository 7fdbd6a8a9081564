"""The allocation-free solver (lbm_solver_create_static): its scratch is the
library's static device array, and it must give exactly the results of
lbm_solver_create with a caller scratch. Two static solvers in a row, the
second on a smaller problem (the array keeps the first one's contents, which
creation clears), each against a regular solver on the same seeded state;
then a problem whose scratch exceeds the array is refused."""
import ctypes

import numpy as np
import pytest

import lbm_workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_08886_amd import lbm
    lbm.lib()


def _pair_of(name, N, nx, ny, nz, storage, layout, seed):
    from paper_1510_08886_amd import lbm
    from tests.parity import dvm_pair
    d, _ = dvm_pair(name)
    prob = lbm.Problem(dim=d.dim, nx=nx, ny=ny, nz=nz, kn=0.07, ma=2e-2, hermite_order=N,
                       storage=storage, layout=layout)
    nodes = nx * ny * (nz if d.dim == 3 else 1)
    rho, u = wl.random_state(nodes, d.dim, seed=seed, amp=1e-2)
    ref = lbm.Solver(d, prob)
    sta = lbm.Solver(d, prob, static_scratch=True)
    for s in (ref, sta):
        s.init(torch.from_numpy(rho), torch.from_numpy(u))
    return ref, sta


@pytest.mark.parametrize("case", [
    # (set, N, nx, ny, nz, storage, layout, steps): the second is smaller
    [("D2V37", 4, 130, 24, 1, "f32", "auto", 37), ("D2V17", 3, 64, 12, 1, "f64", "ping_pong", 20)],
    [("D3V39", 3, 8, 12, 10, "f32", "auto", 9), ("D2V37", 4, 1, 20, 1, "f16dev", "auto", 30)],
])
def test_static_solver_matches_regular_twice(case):
    for k, (name, N, nx, ny, nz, storage, layout, steps) in enumerate(case):
        ref, sta = _pair_of(name, N, nx, ny, nz, storage, layout, seed=17 + k)
        ref.run(steps)
        sta.run(steps)
        assert torch.equal(ref.export(), sta.export()), (name, k)
        a, b = ref.observe(), sta.observe()
        assert a["mdot"] == b["mdot"] and a["mass"] == b["mass"]
        assert torch.equal(a["rho"], b["rho"]) and torch.equal(a["u"], b["u"])
        # a further run continues identically (the partials live in the array)
        ref.run(3)
        sta.run(3)
        assert torch.equal(ref.export(), sta.export()), (name, k)
        ref.close()
        sta.close()


def test_static_solver_refuses_graphs_and_oversized_problems():
    from paper_1510_08886_amd import lbm
    d = lbm.Dvm.named("D2V17")
    s = lbm.Solver(d, lbm.Problem(dim=2, nx=1, ny=40, kn=0.1, hermite_order=3), static_scratch=True)
    with pytest.raises(lbm.LbmError) as err:
        s.set_graph_steps(16)
    assert err.value.code == lbm.LBM_E_UNSUPPORTED
    s.close()
    # a duct whose scratch (wall partials, observation partials) exceeds 16 MiB;
    # the size check comes before any use of the population buffer
    d3 = lbm.Dvm.named("D3V39")
    prob = lbm.Problem(dim=3, nx=64, ny=1024, nz=1024, kn=0.1, hermite_order=3, storage="f32")
    _, scr = lbm.state_bytes(d3, prob)
    assert scr > 16 << 20
    dummy = torch.empty(256, dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    pc = prob.to_c()
    rc = lbm.lib().lbm_solver_create_static(d3._h, ctypes.byref(pc), dummy.data_ptr(),
                                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                            ctypes.byref(h))
    assert rc == -3 and not h.value
    assert b"16 MiB" in lbm.lib().lbm_last_error()
    np.testing.assert_equal(rc, -3)
