"""GPU parity of the Q-method (daq_qmethod_batch through the C ABI) against
the CPU oracle, element by element, bit-exact: the pedestals, the decimated
calorimeter sum (bins of 32 samples) and the fill-by-fill accumulator, over
ragged lengths, several launches into one accumulator, null outputs, both
tile sizes, argument errors and the 16-fill workload at full size."""
import ctypes

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU machines
    pytest.skip("no GPU", allow_module_level=True)

import paper_1611_04959_amd as daq  # noqa: E402
from gpu_util import dev, log, pad_stride, poison  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = daq.Context(0)
    yield c
    c.close()


def _fill(rng, C, N):
    x = rng.integers(-3000, 4000, size=(C, max(N, 1))).astype(np.int16)
    return pad_stride(x[:, :max(N, 1)])


def _check(q, ref_ped, ref_Q, ref_acc, what):
    if q.ped is not None:
        np.testing.assert_array_equal(q.ped.cpu().numpy(), ref_ped, err_msg=what + ": ped")
    if q.qsum is not None:
        np.testing.assert_array_equal(q.qsum.cpu().numpy()[:len(ref_Q)], ref_Q, err_msg=what + ": qsum")
    if q.acc is not None:
        a = q.acc.cpu().numpy()
        np.testing.assert_array_equal(a[:, :ref_acc.shape[1]], ref_acc, err_msg=what + ": acc")


@pytest.mark.parametrize("threads", [256, 512])
def test_random_fills_single_and_batch(ctx, threads):
    ctx.set_schedule(threads, 8, daq.DAQ_VARIANT_SPLIT)
    rng = np.random.default_rng(threads)
    shapes = [(1, 1), (3, 7), (54, 8), (54, 31), (54, 32), (54, 33), (2, 2047), (54, 2048), (5, 2049),
              (54, 4097), (7, 40_000), (54, 0), (1, 100)]
    xs, ns, nps = [], [], []
    for C, N in shapes:
        xs.append(_fill(rng, C, N))
        ns.append(N)
        nps.append(int(rng.integers(1, 150)))
    refs = []
    for x, N, Np in zip(xs, ns, nps):
        acc0 = rng.integers(-10_000, 10_000, size=(x.shape[0], x.shape[1])).astype(np.int32)
        acc = acc0.copy()
        ped, Q = oracle.qmethod(x, N, ped_samples=Np, acc=acc)
        refs.append((acc0, ped, Q, acc))
    fills = [daq.Fill(dev(x), N, ped_samples=Np) for x, N, Np in zip(xs, ns, nps)]
    for mode in ("single", "batch"):
        qs = []
        for f, (acc0, *_r) in zip(fills, refs):
            q = daq.alloc_q_out(f)
            q.acc[:, :acc0.shape[1]] = torch.from_numpy(acc0).cuda()
            qs.append(q)
        log("q-method threads=%d mode=%s" % (threads, mode))
        if mode == "single":
            for f, q in zip(fills, qs):
                ctx.daq_qmethod_batch([f], [q])
        else:
            ctx.daq_qmethod_batch(fills, qs)
        torch.cuda.synchronize()
        for i, (q, (acc0, ped, Q, acc)) in enumerate(zip(qs, refs)):
            _check(q, ped, Q, acc[:, :ns[i]], "fill %d C=%d N=%d %s" % (i, xs[i].shape[0], ns[i], mode))
            # elements past N are never touched
            a = q.acc.cpu().numpy()
            np.testing.assert_array_equal(a[:, ns[i]:acc0.shape[1]], acc0[:, ns[i]:])
    ctx.set_schedule(256, 16, daq.DAQ_VARIANT_SPLIT)


def test_launches_accumulate_in_order_and_wrap(ctx):
    rng = np.random.default_rng(9)
    xa, xb = _fill(rng, 54, 5000), _fill(rng, 54, 5000)
    acc = np.zeros((54, 5000), np.int32)
    acc[0, :4] = [2**31 - 1, -2**31, 2**31 - 5, 7]
    ref = acc.copy()
    oracle.qmethod(xa, 5000, acc=ref)
    _, Qb = oracle.qmethod(xb, 5000, acc=ref)
    f = [daq.Fill(dev(xa), 5000), daq.Fill(dev(xb), 5000)]
    q = daq.alloc_q_out(f[0])
    q.acc[:, :5000] = torch.from_numpy(acc).cuda()
    ctx.daq_qmethod_batch([f[0]], [q])
    ctx.daq_qmethod_batch([f[1]], [q])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(q.acc.cpu().numpy()[:, :5000], ref)
    np.testing.assert_array_equal(q.qsum.cpu().numpy(), Qb)


def test_null_outputs(ctx):
    rng = np.random.default_rng(4)
    x = _fill(rng, 54, 10_000)
    acc = np.zeros((54, 10_000), np.int32)
    ped, Q = oracle.qmethod(x, 10_000, acc=acc)
    f = daq.Fill(dev(x), 10_000)
    only_q = daq.QOut(qsum=poison(torch.empty(len(Q), dtype=torch.int64, device="cuda")))
    only_acc = daq.QOut(acc=torch.zeros((54, 10_000), dtype=torch.int32, device="cuda"))
    only_ped = daq.QOut(ped=poison(torch.empty(54, dtype=torch.int32, device="cuda")))
    f2 = daq.Fill(dev(x), 10_000)
    f3 = daq.Fill(dev(x), 10_000)
    ctx.daq_qmethod_batch([f, f2, f3], [only_q, only_acc, only_ped])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(only_q.qsum.cpu().numpy(), Q)
    np.testing.assert_array_equal(only_acc.acc.cpu().numpy(), acc)
    np.testing.assert_array_equal(only_ped.ped.cpu().numpy(), ped)


def test_argument_errors(ctx):
    lib = daq.load_library()
    x = dev(pad_stride(np.zeros((2, 100), np.int16)))
    f = daq.Fill(x, 100)
    q = daq.alloc_q_out(f)
    fa = (daq.daq_fill * 2)(f.c_struct(), f.c_struct())
    # two fills adding to the same accumulator in one call
    qa = (daq.daq_q_out * 2)(q.c_struct(), q.c_struct())
    assert lib.daq_qmethod_batch(ctx.handle, fa, qa, 2, None) == daq.DAQ_EINVAL
    one = (daq.daq_q_out * 1)()
    one[0] = daq.daq_q_out(None, q.acc.data_ptr(), 96, None)          # stride < N
    assert lib.daq_qmethod_batch(ctx.handle, fa, one, 1, None) == daq.DAQ_EINVAL
    one[0] = daq.daq_q_out(None, q.acc.data_ptr(), 102, None)         # stride % 4 != 0
    assert lib.daq_qmethod_batch(ctx.handle, fa, one, 1, None) == daq.DAQ_EINVAL
    one[0] = daq.daq_q_out(None, q.acc.data_ptr() + 4, 100, None)     # not 16-byte aligned
    assert lib.daq_qmethod_batch(ctx.handle, fa, one, 1, None) == daq.DAQ_EALIGN
    one[0] = daq.daq_q_out(q.qsum.data_ptr() + 4, None, 0, None)      # qsum not 8-byte aligned
    assert lib.daq_qmethod_batch(ctx.handle, fa, one, 1, None) == daq.DAQ_EALIGN
    assert lib.daq_qmethod_batch(None, fa, one, 1, None) == daq.DAQ_EINVAL
    assert lib.daq_qmethod_batch(ctx.handle, fa, one, 0, None) == daq.DAQ_OK


def test_workload_16_fills(ctx):
    """The benchmark batch at full size: 16 fills x 54 ch x 560,000 samples."""
    specs = synth.config_c1()
    xs = synth.render_many(specs)
    fills = [daq.Fill(d, s.n_samples, ped_samples=s.ped_samples) for d, s in zip(synth.to_device(xs), specs)]
    qs = [daq.alloc_q_out(f) for f in fills]
    log("q-method on 16 fills")
    ctx.daq_qmethod_batch(fills, qs)
    ctx.daq_qmethod_batch(fills, qs)    # two fills' worth in every accumulator
    torch.cuda.synchronize()
    for i in (0, 7, 15):
        N = specs[i].n_samples
        acc = np.zeros((54, N), np.int32)
        oracle.qmethod(xs[i], N, ped_samples=specs[i].ped_samples, acc=acc)
        ped, Q = oracle.qmethod(xs[i], N, ped_samples=specs[i].ped_samples, acc=acc)
        _check(qs[i], ped, Q, acc, "fill %d" % i)
