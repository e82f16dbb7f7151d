"""The benchmark's bandwidth reference kernels (libppa_bwprobe.so) move the
bytes they claim: the copy reproduces its input, the read-plus-eighth-write
kernel writes every eighth 16-byte unit of its input, the read visits every
unit exactly once with either workgroup size, and sizes that are not whole
units are refused."""
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
    lib.ppa_probe_read_wg.argtypes = [vp, i64, ci, ci, ci, ci, ctypes.c_uint32, vp, ci, vp]
    lib.ppa_probe_read_streams.argtypes = [vp, i64, ci, ci, ctypes.c_uint32, vp, ci, vp]
    lib.ppa_probe_spmv_mix.argtypes = [vp, vp, vp, vp, i64, i64, ci, ci, ctypes.c_uint32, vp, vp]
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


@pytest.mark.parametrize("threads", [256, 1024])
@pytest.mark.parametrize("contiguous", [0, 1])
@pytest.mark.parametrize("width,nt", [(16, 1), (16, 0), (4, 0)])
def test_read_visits_every_unit_once(probe, width, nt, contiguous, threads):
    """Data zero but for one unit, never = 0: every thread whose XOR is zero
    writes its sink entry, so exactly one entry (the thread that read the
    marked unit, once) keeps its initial value.  Marked units at the start,
    inside and at the end, over ragged sizes and grids."""
    s = torch.cuda.current_stream().cuda_stream
    words_per_unit = width // 4
    for units, blocks in ((1, 0), (1000 + 3, 5), (1 << 16, 0), ((1 << 16) + 17, 256)):
        x = torch.zeros(units * words_per_unit, dtype=torch.int32, device="cuda")
        for mark in sorted({0, units // 2, units - 1}):
            x.zero_()
            x[mark * words_per_unit] = 0x5A5A5A5
            grid = blocks if blocks > 0 else 4096
            sink = torch.full((grid * threads,), -1, dtype=torch.int32, device="cuda")
            rc = probe.ppa_probe_read_wg(x.data_ptr(), units * width, width, nt, contiguous, threads, 0,
                                         sink.data_ptr(), blocks, s)
            assert rc == 0
            torch.cuda.synchronize()
            launched = min(grid, -(-units // threads))
            used = sink[:launched * threads]
            assert int((used == -1).sum()) == 1, (units, blocks, mark)
            assert torch.all(sink[launched * threads:] == -1)


def test_read_workgroup_size_refusals(probe):
    s = torch.cuda.current_stream().cuda_stream
    x = rand_words(1 << 10, 4)
    sink = torch.zeros(4096 * 1024, dtype=torch.int32, device="cuda")
    for threads in (0, 64, 512, 2048):
        assert probe.ppa_probe_read_wg(x.data_ptr(), 4 << 10, 16, 0, 1, threads, 0, sink.data_ptr(), 0, s) == -1


@pytest.mark.parametrize("threads", [256, 1024])
@pytest.mark.parametrize("streams", [1, 2, 4])
def test_read_streams_visits_every_unit_once(probe, streams, threads):
    """As for the single-stream read: one marked 16-byte unit, in the first,
    a middle or the last stream, is read by exactly one thread, once."""
    s = torch.cuda.current_stream().cuda_stream
    for per_stream, blocks in ((1, 0), (1000 + 3, 7), (1 << 15, 256)):
        units = per_stream * streams
        x = torch.zeros(units * 4, dtype=torch.int32, device="cuda")
        for mark in sorted({0, units // 2, units - 1}):
            x.zero_()
            x[4 * mark + 1] = 0x2468ACE
            grid = blocks if blocks > 0 else 4096
            sink = torch.full((grid * threads,), -1, dtype=torch.int32, device="cuda")
            assert probe.ppa_probe_read_streams(x.data_ptr(), 16 * units, streams, threads, 0,
                                                sink.data_ptr(), blocks, s) == 0
            torch.cuda.synchronize()
            launched = min(grid, -(-per_stream // threads))
            assert int((sink[:launched * threads] == -1).sum()) == 1, (per_stream, blocks, mark)
    sink = torch.zeros(4096 * 1024, dtype=torch.int32, device="cuda")
    assert probe.ppa_probe_read_streams(x.data_ptr(), 16 * streams + 16, streams, threads, 0, sink.data_ptr(),
                                        0, s) == (-1 if streams > 1 else 0)
    assert probe.ppa_probe_read_streams(x.data_ptr(), 64, 3, threads, 0, sink.data_ptr(), 0, s) == -1
    assert probe.ppa_probe_read_streams(x.data_ptr(), 64, streams, 512, 0, sink.data_ptr(), 0, s) == -1
    torch.cuda.synchronize()


def test_spmv_mix_stores_every_row_once_per_mode(probe):
    """The sliding-window stream probe: storing per chunk and storing after
    each workgroup's last chunk write the same value to every row, and the
    load-only mode writes none; arguments that do not fit are refused."""
    s = torch.cuda.current_stream().cuda_stream
    chunks, per, rows = 12, 3, 150
    nnz = chunks * 4096
    idx = rand_words(nnz, 11)
    val = rand_words(2 * nnz, 12)
    vec = rand_words(2 * chunks * rows, 13)
    sink = torch.zeros((chunks // per) * 1024, dtype=torch.int32, device="cuda")
    def mix(out_ptr, chunks, per, rows, store):
        return probe.ppa_probe_spmv_mix(idx.data_ptr(), val.data_ptr(), vec.data_ptr(), out_ptr, chunks, per,
                                        rows, store, 0x9E3779B9, sink.data_ptr(), s)

    outs = {}
    for store in (0, 1, 2):
        out = torch.full((2 * chunks * rows,), -5, dtype=torch.int32, device="cuda")
        assert mix(out.data_ptr(), chunks, per, rows, store) == 0
        torch.cuda.synchronize()
        outs[store] = out
    assert torch.all(outs[0] == -5)
    assert torch.equal(outs[1], outs[2])
    pairs = outs[1].view(-1, 2)
    assert torch.all(pairs[:, 1] == ~pairs[:, 0])          # every row written: (acc, ~acc)
    op = outs[0].data_ptr()
    for bad in ((op, chunks, per, 0, 1), (op, chunks, per, 1025, 1), (op, 13, per, rows, 1),
                (op, chunks, per, rows, 3), (op, 60, 60, 150, 2),      # 60 x 150 rows kept: too many
                (op + 8, chunks, per, rows, 1)):                      # output not 16-byte aligned
        assert mix(*bad) == -1
