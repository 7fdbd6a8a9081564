"""The streaming copy used as the bandwidth reference of the benchmark: exact
byte copy through the C ABI, tails of one vector, and argument errors."""
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [16, 4096, 16 * 257, 155_189_248])
def test_stream_copy_is_exact(nbytes):
    from paper_1510_08886_amd import lbm
    g = torch.Generator(device="cuda:0").manual_seed(nbytes)
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda:0", generator=g)
    dst = torch.zeros_like(src)
    lbm.stream_copy(src, dst)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


def test_stream_copy_rejects_unaligned_sizes():
    from paper_1510_08886_amd import lbm
    a = torch.zeros(40, dtype=torch.uint8, device="cuda:0")
    b = torch.zeros_like(a)
    with pytest.raises(lbm.LbmError):
        lbm.stream_copy(a, b)          # 40 bytes: not a multiple of 16
    with pytest.raises(ValueError):
        lbm.stream_copy(a[:32], b[:16])


def test_time_launches_steps_the_solver():
    """lbm_time_launches runs exactly n x steps_per_launch steps (the state
    equals a plain run of as many steps) and returns n positive durations."""
    import lbm_workloads as wl
    from paper_1510_08886_amd import lbm
    d = lbm.Dvm.named("D2V37")
    prob = lbm.Problem(dim=2, nx=128, ny=40, kn=0.1, hermite_order=4, storage="f32")
    rho, u = wl.random_state(128 * 40, 2, seed=4, amp=1e-2)
    a = lbm.Solver(d, prob).init(torch.from_numpy(rho), torch.from_numpy(u))
    b = lbm.Solver(d, prob).init(torch.from_numpy(rho), torch.from_numpy(u))
    for scope in (False, True):
        ms = a.time_launches(5, 1, system_scope=scope)
        assert ms.shape == (5,) and (ms > 0).all() and (ms < 1000).all()
    b.run(10)
    assert a.steps == b.steps == 10
    assert torch.equal(a.export(), b.export())
    with pytest.raises(lbm.LbmError):
        a.time_launches(0)
    a.close()
    b.close()
