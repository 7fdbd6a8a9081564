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
