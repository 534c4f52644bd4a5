"""The read-ceiling kernels read what their declarations say: the XOR of
daq_read_stream's per-wave words is the XOR of every 32-bit word of the
buffer's whole 16-byte words (each read once, either layout), the sum of
daq_read_tiles' per-wave words is the sum over the scan's tiles of the words
each tile covers (halo groups counted once per tile that reads them, island
pattern groups once more in the re-read modes), and the packed write of mode 2
holds each tile's pattern groups in thread order."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU machines
    pytest.skip("no GPU", allow_module_level=True)

import paper_1611_04959_amd as daq  # noqa: E402

OWNED, LEFT, GROUPS = 4048, 32, 512  # the split scan's tile at 512 threads


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("n_words, blocks", [(262_147, 7), (64, 1), (1_000_000, 64)])
def test_read_stream_reads_every_word_once(layout, n_words, blocks):
    rng = np.random.default_rng(n_words + layout)
    x = rng.integers(0, 2**32, size=n_words, dtype=np.uint64).astype(np.uint32)
    buf = torch.from_numpy(x.view(np.int32)).cuda()
    sink = torch.full((blocks * 4,), -1, dtype=torch.int32, device="cuda")
    daq.read_stream(buf, sink, blocks, layout)
    torch.cuda.synchronize()
    got = np.bitwise_xor.reduce(sink.cpu().numpy().view(np.uint32))
    whole = (n_words * 4 // 16) * 4  # 32-bit words of the whole 16-byte words
    assert got == np.bitwise_xor.reduce(x[:whole])


def tile_groups(N):
    """(first group, last group + 1) of each tile's window, clipped to the row."""
    n_groups = N // 8
    out = []
    for lt in range((N + OWNED - 1) // OWNED):
        g0 = (lt * OWNED - LEFT) // 8
        out.append((g0, max(g0, 0), min(g0 + GROUPS, n_groups)))
    return out


def tiles_expected(x, n_fills, C, N, reread=False):
    """Sum over tiles of the 32-bit words of every 8-sample group each tile
    reads (window of 512 groups starting 4 groups before each 506-group
    step); with reread, the groups of the island pattern (group % 70 < 11)
    count once more per tile."""
    words = x.reshape(n_fills, C, N // 8, 4).astype(np.uint64).sum(axis=3)  # per group
    n_groups = N // 8
    count = np.zeros(n_groups, np.uint64)
    pat = (np.arange(n_groups) % 70) < 11
    for _, lo, hi in tile_groups(N):
        count[lo:hi] += 1
        if reread:
            count[lo:hi] += pat[lo:hi].astype(np.uint64)
    return int((words * count[None, None, :]).sum() % (1 << 32))


CASES = [(3, 5, 10_000, 2), (2, 54, 8, 1), (1, 7, 4048 * 3, 3), (4, 13, 33_336, 256)]


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("n_fills, C, N, blocks", CASES)
def test_read_tiles_reads_the_scan_tiles(n_fills, C, N, blocks, mode):
    rng = np.random.default_rng(N + C + mode)
    x = rng.integers(-32768, 32768, size=n_fills * C * N, dtype=np.int64).astype(np.int16)
    raw = torch.from_numpy(x).cuda()
    sink = torch.full((blocks * 8,), -1, dtype=torch.int32, device="cuda")
    tiles = (N + OWNED - 1) // OWNED
    out = None
    if mode == 2:
        out = torch.full((n_fills * tiles * C * 512 * 8,), 0x5A5A, dtype=torch.int16, device="cuda")
    daq.read_tiles(raw, n_fills, C, N, sink, blocks, mode, out)
    torch.cuda.synchronize()
    got = int(sink.cpu().numpy().view(np.uint32).astype(np.uint64).sum() % (1 << 32))
    assert got == tiles_expected(x.view(np.uint32), n_fills, C, N, reread=mode > 0)
    if mode == 2:
        # each tile's pattern groups, in thread order, packed row by row
        o = out.cpu().numpy().reshape(n_fills * tiles, C, 512, 8)
        xr = x.reshape(n_fills, C, N)
        for f in range(n_fills):
            for lt, (g0, lo, hi) in enumerate(tile_groups(N)):
                groups = [g for g in range(lo, hi) if g % 70 < 11]
                t = f * tiles + lt
                for k, g in enumerate(groups):
                    assert np.array_equal(o[t, :, k, :], xr[f, :, 8 * g:8 * g + 8]), (f, lt, k)
                assert (o[t, :, len(groups):, :] == 0x5A5A).all()


def test_read_calls_reject_bad_arguments():
    lib = daq.load_library()
    buf = torch.zeros(1024, dtype=torch.int16, device="cuda")
    sink = torch.zeros(64, dtype=torch.int32, device="cuda")
    assert lib.daq_read_stream(buf.data_ptr(), 8, sink.data_ptr(), 1, 0, None) == daq.DAQ_EINVAL
    assert lib.daq_read_stream(buf.data_ptr(), 2048, sink.data_ptr(), 1, 2, None) == daq.DAQ_EINVAL
    assert lib.daq_read_stream(buf.data_ptr() + 2, 1024, sink.data_ptr(), 1, 0, None) == daq.DAQ_EINVAL
    p, q = buf.data_ptr(), sink.data_ptr()
    assert lib.daq_read_tiles(p, 1, 1, 12, q, 1, 0, None, None) == daq.DAQ_EINVAL
    assert lib.daq_read_tiles(p, 0, 1, 8, q, 1, 0, None, None) == daq.DAQ_EINVAL
    assert lib.daq_read_tiles(p, 1, 1, 8, q, 0, 0, None, None) == daq.DAQ_EINVAL
    assert lib.daq_read_tiles(p + 2, 1, 1, 8, q, 1, 0, None, None) == daq.DAQ_EINVAL
    assert lib.daq_read_tiles(p, 1, 1, 8, q, 1, 3, None, None) == daq.DAQ_EINVAL
    assert lib.daq_read_tiles(p, 1, 1, 8, q, 1, 2, None, None) == daq.DAQ_EINVAL
    assert lib.daq_read_tiles(p, 1, 1, 8, q, 1, 2, p + 2, None) == daq.DAQ_EINVAL
