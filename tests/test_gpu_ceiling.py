"""The read-ceiling kernels read what their declarations say: the XOR of
daq_read_stream's per-wave words is the XOR of every 32-bit word of the
buffer's whole 16-byte words (each read once, either layout), and the sum of
daq_read_tiles' per-wave words is the sum over the scan's tiles of the words
each tile covers (halo groups counted once per tile that reads them)."""
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


def tiles_expected(x, n_fills, C, N):
    """Sum over tiles of the 32-bit words of every 8-sample group each tile
    reads, from the tile geometry (window of 512 groups starting 4 groups
    before each 506-group step)."""
    words = x.reshape(n_fills, C, N // 8, 4).astype(np.uint64).sum(axis=3)  # per group
    n_groups = N // 8
    count = np.zeros(n_groups, np.uint64)
    for lt in range((N + OWNED - 1) // OWNED):
        g0 = (lt * OWNED - LEFT) // 8
        lo, hi = max(g0, 0), min(g0 + GROUPS, n_groups)
        count[lo:hi] += 1
    return int((words * count[None, None, :]).sum() % (1 << 32))


@pytest.mark.parametrize("n_fills, C, N, blocks", [(3, 5, 10_000, 2), (2, 54, 8, 1), (1, 7, 4048 * 3, 3),
                                                   (4, 13, 33_336, 256)])
def test_read_tiles_reads_the_scan_tiles(n_fills, C, N, blocks):
    rng = np.random.default_rng(N + C)
    x = rng.integers(-32768, 32768, size=n_fills * C * N, dtype=np.int64).astype(np.int16)
    raw = torch.from_numpy(x).cuda()
    sink = torch.full((blocks * 8,), -1, dtype=torch.int32, device="cuda")
    daq.read_tiles(raw, n_fills, C, N, sink, blocks)
    torch.cuda.synchronize()
    got = int(sink.cpu().numpy().view(np.uint32).astype(np.uint64).sum() % (1 << 32))
    assert got == tiles_expected(x.view(np.uint32), n_fills, C, N)


def test_read_calls_reject_bad_arguments():
    lib = daq.load_library()
    buf = torch.zeros(1024, dtype=torch.int16, device="cuda")
    sink = torch.zeros(64, dtype=torch.int32, device="cuda")
    assert lib.daq_read_stream(buf.data_ptr(), 8, sink.data_ptr(), 1, 0, None) == daq.DAQ_EINVAL
    assert lib.daq_read_stream(buf.data_ptr(), 2048, sink.data_ptr(), 1, 2, None) == daq.DAQ_EINVAL
    assert lib.daq_read_stream(buf.data_ptr() + 2, 1024, sink.data_ptr(), 1, 0, None) == daq.DAQ_EINVAL
    assert lib.daq_read_tiles(buf.data_ptr(), 1, 1, 12, sink.data_ptr(), 1, None) == daq.DAQ_EINVAL
    assert lib.daq_read_tiles(buf.data_ptr(), 0, 1, 8, sink.data_ptr(), 1, None) == daq.DAQ_EINVAL
    assert lib.daq_read_tiles(buf.data_ptr(), 1, 1, 8, sink.data_ptr(), 0, None) == daq.DAQ_EINVAL
    assert lib.daq_read_tiles(buf.data_ptr() + 2, 1, 1, 8, sink.data_ptr(), 1, None) == daq.DAQ_EINVAL
