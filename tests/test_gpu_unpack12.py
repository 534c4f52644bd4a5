"""GPU parity of the 12-bit ingest (daq_unpack12 through the C ABI) against
the CPU oracle and the original samples, bit-exact, over ragged lengths and
padded strides, argument errors, and a fill unpacked on the device and then
chopped, against the oracle's chop of the original samples."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU machines
    pytest.skip("no GPU", allow_module_level=True)

import paper_1611_04959_amd as daq  # noqa: E402
from gpu_util import assert_same, dev, log  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = daq.Context(0)
    yield c
    c.close()


def pack12(x, stride=None):
    """Vectorised packer from the layout (pairs of samples to three bytes)."""
    C, n = x.shape
    nb = oracle.packed12_row_bytes(n)
    st = nb if stride is None else stride
    v = x.astype(np.uint32) & 0xFFF
    if n % 2:
        v = np.concatenate([v, np.zeros((C, 1), np.uint32)], axis=1)
    a, b = v[:, 0::2], v[:, 1::2]
    trip = np.stack([a & 0xFF, (a >> 8) | ((b & 0xF) << 4), b >> 4], axis=2).reshape(C, -1).astype(np.uint8)
    out = np.zeros((C, max(st, 4)), np.uint8)
    out[:, :nb] = trip[:, :nb]
    return out


@pytest.mark.parametrize("C,n", [(1, 1), (1, 7), (3, 8), (3, 9), (2, 15), (54, 16), (54, 17), (5, 1001),
                                 (54, 560_000), (2, 0)])
def test_unpack_matches(ctx, C, n):
    rng = np.random.default_rng(C * 1000 + n)
    x = rng.integers(0, 4096, size=(C, max(n, 1))).astype(np.int16)[:, :n]
    stride = (oracle.packed12_row_bytes(n) + 3) // 4 * 4 + 8           # padded packed rows
    p = pack12(x, stride)
    assert (oracle.unpack12(p, n) == x).all()
    raw = torch.full((C, max(daq.padded(n), 8) + 8), -7, dtype=torch.int16, device="cuda")
    log("unpack12 C=%d n=%d" % (C, n))
    ctx.daq_unpack12(dev(p), n, raw)
    torch.cuda.synchronize()
    got = raw.cpu().numpy()
    np.testing.assert_array_equal(got[:, :n], x)
    assert (got[:, n:] == -7).all()   # samples >= n untouched


def test_argument_errors(ctx):
    lib = daq.load_library()
    p = torch.zeros((2, 16), dtype=torch.uint8, device="cuda")
    r = torch.zeros((2, 16), dtype=torch.int16, device="cuda")
    h = ctx.handle
    assert lib.daq_unpack12(h, p.data_ptr(), 16, 2, 11, r.data_ptr(), 16, None) == daq.DAQ_EINVAL   # 17 bytes > 16
    assert lib.daq_unpack12(h, p.data_ptr(), 16, 2, 10, r.data_ptr(), 8, None) == daq.DAQ_EINVAL   # stride < n
    assert lib.daq_unpack12(h, p.data_ptr() + 1, 16, 2, 10, r.data_ptr(), 16, None) == daq.DAQ_EALIGN
    assert lib.daq_unpack12(h, p.data_ptr(), 15, 1, 10, r.data_ptr(), 16, None) == daq.DAQ_EALIGN
    assert lib.daq_unpack12(h, p.data_ptr(), 16, 2, 10, r.data_ptr() + 2, 16, None) == daq.DAQ_EALIGN
    assert lib.daq_unpack12(h, p.data_ptr(), 16, 0, 10, r.data_ptr(), 16, None) == daq.DAQ_EINVAL
    assert lib.daq_unpack12(None, p.data_ptr(), 16, 2, 10, r.data_ptr(), 16, None) == daq.DAQ_EINVAL
    assert lib.daq_unpack12(h, p.data_ptr(), 16, 2, 0, r.data_ptr(), 16, None) == daq.DAQ_OK


def test_unpack_then_chop(ctx):
    """A plain-workload fill arriving as 12-bit words: unpacked and chopped on the device."""
    spec = synth.config_c0()[0]
    x = synth.render(spec)                    # int16 [54, padded N], 12-bit values
    N = spec.n_samples
    assert x.min() >= 0 and x.max() <= 4095
    p = pack12(x[:, :N], (oracle.packed12_row_bytes(N) + 3) // 4 * 4)
    raw = torch.zeros((x.shape[0], x.shape[1]), dtype=torch.int16, device="cuda")
    ctx.daq_unpack12(dev(p), N, raw)
    f = daq.Fill(raw, N, threshold=spec.threshold, pre=spec.pre, post=spec.post, ped_samples=spec.ped_samples)
    fo = daq.alloc_out(f)
    ctx.daq_chop_fill(f, fo)
    torch.cuda.synchronize()
    ref = oracle.chop(x, n_samples=N, ped_samples=spec.ped_samples, threshold=spec.threshold,
                      pre=spec.pre, post=spec.post)
    assert_same(fo, ref, ctx="unpacked fill")
