"""GPU test of daq_process_batch_noalloc (the entry point for callers that
cannot allocate): through the C ABI, its results equal daq_process_batch's
on the same fills, element by element, on two calls in a row (the second
with a smaller batch), and equal the CPU oracle; a batch too large for the
static scratch is refused before anything runs."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU machines
    pytest.skip("no GPU", allow_module_level=True)

import paper_1611_04959_amd as daq  # noqa: E402
from gpu_util import assert_same, dev, log, make_fill, oracle_many, pad_stride, poison_out  # noqa: E402


def _fills(rng, n, n_lo, n_hi):
    xs, ns, ps = [], [], []
    for _ in range(n):
        N = int(rng.integers(n_lo, n_hi))
        x = rng.integers(995, 1006, size=(54, N)).astype(np.int16)
        for _ in range(int(rng.integers(1, max(2, N // 500)))):
            t = int(rng.integers(0, N))
            x[rng.integers(0, 54), t:t + int(rng.integers(1, 30))] -= np.int16(rng.integers(0, 500))
        xs.append(pad_stride(x))
        ns.append(N)
        ps.append({"threshold": int(rng.integers(-300, -60)), "pre": int(rng.integers(0, 20)),
                   "post": int(rng.integers(0, 50)), "ped_samples": int(rng.integers(1, 150))})
    return xs, ns, ps


def _compare(a, b, what):
    ia, na, ta, sa, pa, oa = a.host()
    ib, nb, tb, sb, pb, ob = b.host()
    assert (na, ta, sa) == (nb, tb, sb), what
    np.testing.assert_array_equal(ia, ib, err_msg=what + ": records")
    np.testing.assert_array_equal(pa, pb, err_msg=what + ": pedestals")
    np.testing.assert_array_equal(oa, ob, err_msg=what + ": packed rows")


def test_noalloc_equals_process_batch_twice():
    rng = np.random.default_rng(2024)
    with daq.Context(0) as ctx:
        # a full-size calorimeter fill among ragged small ones, then a smaller batch
        spec = synth.config_c1(1)[0]
        big = synth.render(spec)
        p_big = {"threshold": spec.threshold, "pre": spec.pre, "post": spec.post, "ped_samples": spec.ped_samples}
        xs, ns, ps = _fills(rng, 7, 1, 40_000)
        batches = [([big] + xs, [spec.n_samples] + ns, [p_big] + ps)]
        xs2, ns2, ps2 = _fills(rng, 3, 1, 9_000)
        batches.append((xs2, ns2, ps2))
        for call, (bx, bn, bp) in enumerate(batches):
            refs = oracle_many(bx, bn, bp)
            fills = [make_fill(dev(x), n, p) for x, n, p in zip(bx, bn, bp)]
            need = daq.noalloc_scratch_bytes(fills)
            log("noalloc call %d: %d fills, %d scratch bytes" % (call, len(fills), need))
            assert 0 < need <= daq.DAQ_NOALLOC_SCRATCH_BYTES
            want = [daq.alloc_out(f) for f in fills]
            got = [daq.alloc_out(f) for f in fills]
            ctx.daq_process_batch(fills, want)
            for o in got:
                poison_out(o)
            torch.cuda.synchronize()
            ctx.daq_process_batch_noalloc(fills, got)
            torch.cuda.synchronize()
            for i, (g, w, r) in enumerate(zip(got, want, refs)):
                _compare(g, w, "call %d fill %d" % (call, i))
                assert_same(g, r, ctx="call %d fill %d vs oracle" % (call, i))


def test_noalloc_refuses_what_does_not_fit():
    with daq.Context(0) as ctx:
        x = torch.zeros((54, 8), dtype=torch.int16, device="cuda")
        # 64 fills of 54 x 2,000,000 samples need far more than the static
        # scratch: refused on the host before anything is launched
        lib = daq.load_library()
        fa = (daq.daq_fill * 64)()
        for i in range(64):
            fa[i] = daq.daq_fill(x.data_ptr(), 2_000_000, 2_000_000, 54, 100, -200, 8, 24, 0)
        assert lib.daq_noalloc_scratch_bytes(fa, 64) > daq.DAQ_NOALLOC_SCRATCH_BYTES
        oa = (daq.daq_fill_out * 64)()
        cnt = torch.zeros(3, dtype=torch.int64, device="cuda")
        for i in range(64):
            oa[i] = daq.daq_fill_out(None, 0, cnt.data_ptr(), None, None, 0)
        assert lib.daq_process_batch_noalloc(ctx.handle, fa, oa, 64, None) == daq.DAQ_ERANGE
        assert lib.daq_process_batch_noalloc(ctx.handle, fa, oa, 0, None) == daq.DAQ_OK
        assert lib.daq_process_batch_noalloc(None, fa, oa, 1, None) == daq.DAQ_EINVAL
