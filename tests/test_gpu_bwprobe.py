"""The benchmark's bandwidth reference kernels (libppa_bwprobe.so) move the
bytes they claim: the copy reproduces its input, the read-plus-eighth-write
kernel writes every eighth 16-byte unit of its input, and sizes that are not
whole units are refused."""
import ctypes
import os

import pytest
import torch

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROBE = os.path.join(ROOT, "paper_1806_08020_amd", "libppa_bwprobe.so")


@pytest.fixture(scope="module")
def probe():
    if not os.path.exists(PROBE):
        pytest.fail("libppa_bwprobe.so is not built (run python -m paper_1806_08020_amd.build)")
    lib = ctypes.CDLL(PROBE)
    vp, i64, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.ppa_probe_read.argtypes = [vp, i64, ci, ci, ci, ctypes.c_uint32, vp, ci, vp]
    lib.ppa_probe_copy.argtypes = [vp, vp, i64, ci, ci, vp]
    lib.ppa_probe_read_write8.argtypes = [vp, vp, i64, ci, ci, vp]
    return lib


def rand_words(n, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    return torch.randint(-2 ** 31, 2 ** 31 - 1, (n,), dtype=torch.int32, device="cuda", generator=g)


@pytest.mark.parametrize("contiguous", [0, 1])
@pytest.mark.parametrize("words,blocks", [(4, 0), (4 * 1000 + 4, 7), (1 << 20, 0), ((1 << 20) + 12, 3)])
def test_copy(probe, words, blocks, contiguous):
    s = torch.cuda.current_stream().cuda_stream
    x = rand_words(words, words)
    y = torch.full_like(x, -1)
    assert probe.ppa_probe_copy(x.data_ptr(), y.data_ptr(), 4 * words, contiguous, blocks, s) == 0
    torch.cuda.synchronize()
    assert torch.equal(x, y)


@pytest.mark.parametrize("contiguous", [0, 1])
@pytest.mark.parametrize("units,blocks", [(8, 0), (8 * 1001, 5), (1 << 18, 0)])
def test_read_write_eighth(probe, units, blocks, contiguous):
    s = torch.cuda.current_stream().cuda_stream
    x = rand_words(4 * units, units + 1)
    y = torch.full((units // 8 + 1, 4), -7, dtype=torch.int32, device="cuda")
    assert probe.ppa_probe_read_write8(x.data_ptr(), y.data_ptr(), 16 * units, contiguous, blocks, s) == 0
    torch.cuda.synchronize()
    want = x.view(units, 4)[::8]
    assert torch.equal(y[:units // 8], want)
    assert torch.all(y[units // 8] == -7)          # nothing written past bytes / 8


def test_read_runs_and_refusals(probe):
    s = torch.cuda.current_stream().cuda_stream
    x = rand_words(1 << 16, 3)
    sink = torch.zeros(4096 * 256, dtype=torch.int32, device="cuda")
    xp, sp = x.data_ptr(), sink.data_ptr()
    for width, nt in ((16, 1), (16, 0), (4, 0)):
        for contiguous in (0, 1):
            assert probe.ppa_probe_read(xp, 4 << 16, width, nt, contiguous, 0x9E3779B9, sp, 0, s) == 0
    assert probe.ppa_probe_read(xp, 0, 16, 0, 0, 0, sp, 0, s) == 0
    torch.cuda.synchronize()
    assert probe.ppa_probe_read(xp, 20, 16, 0, 0, 0, sp, 0, s) == -1       # not whole 16-byte units
    assert probe.ppa_probe_read(xp, 64, 8, 0, 0, 0, sp, 0, s) == -1        # width 8 is not offered
    assert probe.ppa_probe_read(xp, 64, 4, 1, 0, 0, sp, 0, s) == -1        # non-temporal only at 16 bytes
    assert probe.ppa_probe_copy(xp, xp, 24, 0, 0, s) == -1
    assert probe.ppa_probe_read_write8(xp, xp, 64, 0, 0, s) == -1          # not whole 128-byte pieces
