"""GPU parity of the island compression (daq_compress_batch through the C ABI)
against the CPU oracle, bit-exact: block headers, payload words, stream
length and block offsets, over ragged row lengths (short last blocks, rows of
one sample, empty streams), extreme differences (17-bit codes), flat rows
(empty payloads), batches past one launch's fill count, a cut-short stream,
max_len clamping, argument errors, 40 fills of random shape in one call, and
the 16-fill workload chopped on the device and then compressed, decoded back
to the oracle's packed samples."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU machines
    pytest.skip("no GPU", allow_module_level=True)

import paper_1611_04959_amd as daq  # noqa: E402
from gpu_util import dev, log, make_fill, oracle_many, poison  # noqa: E402
from test_gpu_parity import params  # noqa: E402

B = oracle.Z_BLOCK


@pytest.fixture(scope="module")
def ctx():
    c = daq.Context(0)
    yield c
    c.close()


def rows(seed, C, L, kind):
    """int16 [C, L] rows: 'noise' (a pedestal with small steps), 'wide' (any
    int16), 'flat', 'mixed' (each 64-sample block one of the three)."""
    rng = np.random.default_rng(seed)
    n = max(L, 1)
    if kind == "noise":
        x = 1800 + rng.integers(-6, 7, size=(C, n))
    elif kind == "wide":
        x = rng.integers(-32768, 32768, size=(C, n))
    elif kind == "flat":
        x = np.full((C, n), int(rng.integers(-32768, 32768)))
    elif kind == "mixed":
        x = np.empty((C, n), np.int64)
        for c in range(C):
            for k in range(0, n, B):
                m = min(B, n - k)
                pick = int(rng.integers(0, 4))
                if pick == 0:
                    x[c, k:k + m] = rng.integers(-32768, 32768, size=m)
                elif pick == 1:
                    x[c, k:k + m] = 1700 + rng.integers(-3, 4, size=m)
                elif pick == 2:
                    x[c, k:k + m] = rng.integers(-1000, 1000)
                else:  # the two extremes alternating: 17-bit codes
                    x[c, k:k + m] = np.where(np.arange(m) % 2, 32767, -32768)
    else:
        raise ValueError(kind)
    return x.astype(np.int16)[:, :L]


def packed_out(x, L, extra=0, fill=-5):
    """A FillOut holding x as its packed rows and total_len = L (rows padded
    with `fill` past L, stride a multiple of 8 plus `extra`)."""
    C = x.shape[0]
    st = max(daq.padded(x.shape[1]), 8) + extra
    host = np.full((C, st), fill, np.int16)
    host[:, :x.shape[1]] = x
    counts = torch.tensor([0, L, 0], dtype=torch.int64, device="cuda")
    return daq.FillOut(None, counts, None, dev(host))


def check(zo, x, L, ctx_msg=""):
    C = x.shape[0]
    hdr_ref, words_ref = oracle.z_compress(x, L)
    hdr, offs, words = zo.host(C, L)
    assert int(zo.n_words.item()) == len(words_ref), ctx_msg
    np.testing.assert_array_equal(hdr, hdr_ref, err_msg=ctx_msg + ": headers")
    np.testing.assert_array_equal(words, words_ref, err_msg=ctx_msg + ": payload words")
    if offs is not None:
        # block b's payload starts where the sizes of the blocks before it end
        n = np.array([min(B, L - (b % max(-(-L // B), 1)) * B) for b in range(len(hdr_ref))], np.int64)
        w = (hdr_ref >> 16).astype(np.int64)
        sizes = ((n - 1) * w + 31) // 32
        np.testing.assert_array_equal(offs, np.concatenate([[0], np.cumsum(sizes)[:-1]])[:len(offs)],
                                      err_msg=ctx_msg + ": block offsets")
    np.testing.assert_array_equal(oracle.z_decompress(hdr, words, C, L), x[:, :L], err_msg=ctx_msg + ": decode")


@pytest.mark.parametrize("C,L", [(1, 0), (1, 1), (1, 2), (3, 63), (3, 64), (3, 65), (2, 511), (2, 512),
                                 (2, 513), (54, 1000), (5, 4097), (54, 61_000)])
@pytest.mark.parametrize("kind", ["noise", "wide", "flat", "mixed"])
def test_compress_matches(ctx, C, L, kind):
    x = rows(C * 7919 + L * 31 + len(kind), C, L, kind)
    o = packed_out(x, L, extra=8 if L % 2 else 0)
    zo = daq.alloc_z_out(C, o.out.shape[1], device="cuda")
    log("compress C=%d L=%d %s" % (C, L, kind))
    ctx.daq_compress_batch([o], [zo])
    torch.cuda.synchronize()
    check(zo, x, L, "C=%d L=%d %s" % (C, L, kind))


def test_batch_past_one_launch(ctx):
    """20 fills of different shapes in one call (two launches of the kernels)."""
    xs, outs, zouts, Ls = [], [], [], []
    for i in range(20):
        C, L = 1 + i % 5, 37 * i + (i % 3) * 64
        x = rows(100 + i, C, L, ["noise", "wide", "mixed", "flat"][i % 4])
        xs.append(x)
        Ls.append(L)
        outs.append(packed_out(x, L))
        zouts.append(daq.alloc_z_out(C, outs[-1].out.shape[1], offsets=(i % 2 == 0), device="cuda"))
    log("compress batch of 20")
    ctx.daq_compress_batch(outs, zouts)
    torch.cuda.synchronize()
    for i in range(20):
        check(zouts[i], xs[i], Ls[i], "fill %d" % i)


def test_calls_in_a_row_reuse_scratch(ctx):
    """A large call, then a smaller one on the same stream, both exact."""
    for C, L in [(54, 30_000), (3, 700)]:
        x = rows(C + L, C, L, "mixed")
        o = packed_out(x, L)
        zo = daq.alloc_z_out(C, o.out.shape[1], device="cuda")
        ctx.daq_compress_batch([o], [zo])
        torch.cuda.synchronize()
        check(zo, x, L, "C=%d L=%d" % (C, L))


def test_stream_cut_short(ctx):
    """words_cap below the stream: the length is still reported and no word
    past the cap is written."""
    C, L = 4, 3000
    x = rows(5, C, L, "wide")
    hdr_ref, words_ref = oracle.z_compress(x, L)
    cap = len(words_ref) // 3
    o = packed_out(x, L)
    zo = daq.alloc_z_out(C, o.out.shape[1], device="cuda")
    zo.words.fill_(-1)
    ctx.daq_compress_batch([o], [zo], words_cap=[cap])
    torch.cuda.synchronize()
    assert int(zo.n_words.item()) == len(words_ref)
    w = zo.words.cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(w[:cap], words_ref[:cap])
    assert (w[cap:] == 0xFFFFFFFF).all()
    np.testing.assert_array_equal(zo.hdr[:len(hdr_ref)].cpu().numpy().view(np.uint32), hdr_ref)


def test_max_len_clamps_total_len(ctx):
    """total_len above max_len: only max_len samples of each row are taken."""
    C, L = 3, 900
    x = rows(9, C, L, "noise")
    o = packed_out(x, 5000)               # total_len claims more than the rows hold
    zo = daq.alloc_z_out(C, L, device="cuda")
    ctx.daq_compress_batch([o], [zo], max_len=L)
    torch.cuda.synchronize()
    check(zo, x, L, "clamped")
    # a negative total_len compresses nothing
    o2 = packed_out(x, -3)
    zo2 = daq.alloc_z_out(C, L, device="cuda")
    zo2.n_words.fill_(99)
    ctx.daq_compress_batch([o2], [zo2], max_len=L)
    torch.cuda.synchronize()
    assert int(zo2.n_words.item()) == 0


def test_argument_errors(ctx):
    lib = daq.load_library()
    C, L = 2, 100
    x = rows(1, C, L, "noise")
    o = packed_out(x, L)
    zo = daq.alloc_z_out(C, o.out.shape[1], device="cuda")

    def call(**kw):
        f = daq.daq_z_fill(o.out.data_ptr(), int(o.out.stride(0)), o.counts.data_ptr(), L, zo.hdr.data_ptr(),
                           zo.offsets.data_ptr(), zo.words.data_ptr(), int(zo.words.numel()),
                           zo.n_words.data_ptr(), C, 0)
        for k, v in kw.items():
            setattr(f, k, v)
        arr = (daq.daq_z_fill * 1)(f)
        return lib.daq_compress_batch(ctx.handle, arr, 1, None)

    assert call() == daq.DAQ_OK
    torch.cuda.synchronize()
    assert call(packed=None) == daq.DAQ_EINVAL
    assert call(counts=None) == daq.DAQ_EINVAL
    assert call(hdr=None) == daq.DAQ_EINVAL
    assert call(n_words=None) == daq.DAQ_EINVAL
    assert call(n_channels=0) == daq.DAQ_EINVAL
    assert call(reserved=1) == daq.DAQ_EINVAL
    assert call(max_len=-1) == daq.DAQ_EINVAL
    assert call(max_len=int(o.out.stride(0)) + 1) == daq.DAQ_EINVAL       # rows shorter than max_len
    assert call(n_channels=daq.DAQ_MAX_CHANNELS + 1) == daq.DAQ_ERANGE
    assert call(packed=o.out.data_ptr() + 2) == daq.DAQ_EALIGN
    assert call(stride=int(o.out.stride(0)) - 4) == daq.DAQ_EALIGN
    assert call(offsets=zo.offsets.data_ptr() + 4) == daq.DAQ_EALIGN
    assert lib.daq_compress_batch(ctx.handle, None, 1, None) == daq.DAQ_EINVAL
    assert lib.daq_compress_batch(ctx.handle, None, 0, None) == daq.DAQ_OK
    assert lib.daq_compress_batch(ctx.handle, None, -1, None) == daq.DAQ_EINVAL


def test_workload_16_fills_chopped_then_compressed(ctx):
    """The benchmark's 16 fills chopped in one batched launch, then compressed
    in one call: each stream equals the oracle's compression of the oracle's
    packed samples and decodes back to them."""
    specs = synth.config_c1()
    xs = synth.render_many(specs)
    ns = [s.n_samples for s in specs]
    ps = [params(s.threshold, s.pre, s.post, s.ped_samples) for s in specs]
    refs = oracle_many(xs, ns, ps)
    fills = [make_fill(d, n, p) for d, n, p in zip(synth.to_device(xs), ns, ps)]
    outs = [daq.alloc_out(f) for f in fills]
    zouts = [daq.alloc_z_out(o.out.shape[0], o.out.shape[1], device="cuda") for o in outs]
    log("chop + compress 16 fills")
    ctx.daq_process_batch(fills, outs)
    ctx.daq_compress_batch(outs, zouts)
    torch.cuda.synchronize()
    raw_words = 0
    for i, (zo, r) in enumerate(zip(zouts, refs)):
        check(zo, r.out, r.total_len, "fill %d" % i)
        raw_words += r.out.shape[0] * r.total_len / 2
    ratio = raw_words / sum(int(z.n_words.item()) for z in zouts)
    log("compression ratio %.2f" % ratio)
    assert ratio > 1.5


def test_random_shapes_in_one_call(ctx):
    """40 fills of random shape and content in one call (three launches):
    channel counts 1..70, lengths 0..5000, padded strides, max_len above the
    length, and a mix of the row kinds above."""
    rng = np.random.default_rng(2024)
    xs, Ls, outs, zouts = [], [], [], []
    kinds = ["noise", "wide", "flat", "mixed"]
    for i in range(40):
        C, L = int(rng.integers(1, 71)), int(rng.integers(0, 5001))
        x = rows(5000 + i, C, L, kinds[int(rng.integers(0, 4))])
        o = packed_out(x, L, extra=8 * int(rng.integers(0, 3)))
        xs.append(x)
        Ls.append(L)
        outs.append(o)
        zouts.append(daq.alloc_z_out(C, int(o.out.shape[1]), offsets=bool(i % 3), device="cuda"))
    log("compress 40 random fills")
    ctx.daq_compress_batch(outs, zouts)
    torch.cuda.synchronize()
    for i in range(40):
        check(zouts[i], xs[i], Ls[i], "random fill %d (C=%d L=%d)" % (i, xs[i].shape[0], Ls[i]))


def _offsets_of(hdr, C, L):
    """Payload offsets from the headers (the format's size rule)."""
    nb = -(-L // B)
    n = np.array([min(B, L - (b % max(nb, 1)) * B) for b in range(len(hdr))], np.int64)
    sizes = ((n - 1) * (hdr >> 16).astype(np.int64) + 31) // 32
    return np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64) if len(hdr) else np.zeros(0, np.int64)


@pytest.mark.parametrize("C,L", [(1, 1), (3, 63), (3, 65), (2, 513), (54, 1000), (5, 4097)])
@pytest.mark.parametrize("kind", ["noise", "wide", "flat", "mixed"])
def test_decompress_round_trip(ctx, C, L, kind):
    """Compressed on the device, decoded on the device: the packed rows come
    back exactly, samples past L untouched. The oracle's own stream decodes
    the same way."""
    x = rows(C * 131 + L + len(kind), C, L, kind)
    o = packed_out(x, L)
    zo = daq.alloc_z_out(C, o.out.shape[1], device="cuda")
    ctx.daq_compress_batch([o], [zo])
    back = torch.full((C, max(daq.padded(L), 8) + 8), -3, dtype=torch.int16, device="cuda")
    log("decompress C=%d L=%d %s" % (C, L, kind))
    ctx.daq_decompress_batch([zo], [L], [back])
    torch.cuda.synchronize()
    got = back.cpu().numpy()
    np.testing.assert_array_equal(got[:, :L], x[:, :L])
    assert (got[:, L:] == -3).all()
    # the oracle's stream, decoded by the device
    hdr, words = oracle.z_compress(x, L)
    z2 = daq.ZOut(dev(hdr.view(np.int32) if len(hdr) else np.zeros(1, np.int32)),
                  dev(_offsets_of(hdr, C, L) if len(hdr) else np.zeros(1, np.int64)),
                  dev(words.view(np.int32) if len(words) else np.zeros(1, np.int32)),
                  torch.tensor([len(words)], dtype=torch.int64, device="cuda"))
    back2 = torch.full_like(back, -3)
    ctx.daq_decompress_batch([z2], [L], [back2])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(back2.cpu().numpy()[:, :L], x[:, :L])


def test_decompress_16_fills_and_damaged_streams(ctx):
    """The 16 benchmark fills chopped, compressed and decoded in one call each
    (bit-exact against the packed rows); then streams cut short or with
    widths past 17 decode without error (samples unspecified)."""
    specs = synth.config_c1()
    xs = synth.render_many(specs)
    ns = [s.n_samples for s in specs]
    ps = [params(s.threshold, s.pre, s.post, s.ped_samples) for s in specs]
    fills = [make_fill(d, n, p) for d, n, p in zip(synth.to_device(xs), ns, ps)]
    outs = [daq.alloc_out(f) for f in fills]
    zouts = [daq.alloc_z_out(o.out.shape[0], o.out.shape[1], device="cuda") for o in outs]
    ctx.daq_process_batch(fills, outs)
    ctx.daq_compress_batch(outs, zouts)
    torch.cuda.synchronize()
    Ls = [int(o.counts[1].item()) for o in outs]
    backs = [poison(torch.empty_like(o.out)) for o in outs]
    log("decompress 16 fills")
    ctx.daq_decompress_batch(zouts, Ls, backs)
    torch.cuda.synchronize()
    for i, (o, bk, L) in enumerate(zip(outs, backs, Ls)):
        assert torch.equal(bk[:, :L], o.out[:, :L]), i
    # damaged: the stream cut to half its words, and every header's width field set to 31
    z = zouts[0]
    half = int(z.n_words.item()) // 2
    cut = daq.ZOut(z.hdr, z.offsets, z.words[:half].clone(), z.n_words)
    ctx.daq_decompress_batch([cut], [Ls[0]], [backs[0]])
    z.hdr.bitwise_or_(0x1F << 16)
    ctx.daq_decompress_batch([z], [Ls[0]], [backs[0]])
    torch.cuda.synchronize()


def test_decompress_argument_errors(ctx):
    lib = daq.load_library()
    C, L = 2, 100
    x = rows(3, C, L, "noise")
    o = packed_out(x, L)
    zo = daq.alloc_z_out(C, o.out.shape[1], device="cuda")
    back = torch.zeros((C, 104), dtype=torch.int16, device="cuda")

    def call(**kw):
        s = daq.daq_z_stream(zo.hdr.data_ptr(), zo.offsets.data_ptr(), zo.words.data_ptr(), 10,
                             back.data_ptr(), 104, L, C, 0)
        for k, v in kw.items():
            setattr(s, k, v)
        return lib.daq_decompress_batch(ctx.handle, (daq.daq_z_stream * 1)(s), 1, None)

    assert call() == daq.DAQ_OK
    torch.cuda.synchronize()
    assert call(offsets=None) == daq.DAQ_EINVAL
    assert call(hdr=None) == daq.DAQ_EINVAL
    assert call(out_stride=99) == daq.DAQ_EINVAL
    assert call(reserved=2) == daq.DAQ_EINVAL
    assert call(n_channels=0) == daq.DAQ_EINVAL
    assert call(out=back.data_ptr() + 2) == daq.DAQ_EALIGN
    assert call(out_stride=108) == daq.DAQ_EALIGN
    assert lib.daq_decompress_batch(ctx.handle, None, 0, None) == daq.DAQ_OK
