"""The calibration kernels behind the benchmark's measured peaks do what
their rates are quoted for: the copy moves every byte, and the atomic
patterns add exactly once per operation to the words they name (the
scatter pattern is a bijection, so every word of the range gets one add)."""
import pytest
import torch

from paper_2309_16818_amd import mem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [16, 4096 + 48, (64 << 20) + 16 * 1001])
def test_copy_moves_every_byte(nbytes):
    g = torch.Generator(device="cuda").manual_seed(nbytes)
    src = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device="cuda", generator=g)
    dst = torch.zeros(nbytes + 64, dtype=torch.uint8, device="cuda")
    mem.calib_copy(src, dst[:nbytes])
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src)
    assert not dst[nbytes:].any()


@pytest.mark.parametrize("dtype", [torch.int32, torch.float32])
def test_atomic_patterns_add_once_per_operation(dtype):
    n = 1 << 20
    buf = torch.zeros(n + 256, dtype=dtype, device="cuda")
    mem.calib_atomic(buf, mem.MEM_CALIB_UNIQUE, n - 5, n)
    torch.cuda.synchronize()
    assert (buf[:n - 5] == 1).all() and not buf[n - 5:].any()
    buf.zero_()
    mem.calib_atomic(buf, mem.MEM_CALIB_SCATTER, n, n)
    torch.cuda.synchronize()
    assert (buf[:n] == 1).all() and not buf[n:].any()
    buf.zero_()
    mem.calib_atomic(buf, mem.MEM_CALIB_SCATTER, 1000, 1 << 10)  # a prefix: 1000 distinct words
    torch.cuda.synchronize()
    assert int(buf.sum().item()) == 1000 and int(buf.max().item()) == 1
    buf.zero_()
    mem.calib_atomic(buf, mem.MEM_CALIB_SHARED, 64 * 4096, 64)
    torch.cuda.synchronize()
    assert (buf[:64] == 4096).all() and not buf[64:].any()


def test_gather_loads_every_word_of_its_range_once():
    """With n_lanes x per_lane = n_words the loads visit every word once (the
    scatter bijection); with a table of ones every lane sums per_lane."""
    bits = 16
    n = 1 << bits
    tab = (torch.arange(n, device="cuda") % 7).float()
    out = torch.full((n // 64,), -1.0, device="cuda")
    mem.calib_gather(tab, out, 64)
    torch.cuda.synchronize()
    assert float(out.double().sum().item()) == float((torch.arange(n) % 7).sum().item())
    ones = torch.ones(1 << 18, device="cuda")
    out = torch.zeros(3000, device="cuda")
    mem.calib_gather(ones, out, 40)
    torch.cuda.synchronize()
    assert (out == 40).all()
    out.zero_()
    mem.calib_gather(ones, out, 40, runs=True)
    torch.cuda.synchronize()
    assert (out == 40).all()
    out = torch.full((n // 64,), -1.0, device="cuda")
    mem.calib_gather(tab, out, 64, runs=True)  # runs wrap around the table
    torch.cuda.synchronize()
    assert (out >= 0).all()
    with pytest.raises(mem.MemError):
        mem.calib_gather(ones[:1000], out, 40)  # not a power of two
    with pytest.raises(mem.MemError):
        mem.calib_gather(ones, out, 12)  # not a multiple of 8
