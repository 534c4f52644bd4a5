"""GPU parity of both methods on one read (daq_process_batch_q through the C
ABI): the T-method's island tables, pedestals and packed samples equal the
oracle's chop, and the Q-method's decimated sums and accumulators equal the
oracle's Q-method, bit-exact, over ragged lengths and channel counts, both
tile sizes, a batch cut into fill groups on several streams, a context on
another schedule, where the pedestals go, argument
errors, and the 16-fill workload (also against the two separate calls)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU machines
    pytest.skip("no GPU", allow_module_level=True)

import paper_1611_04959_amd as daq  # noqa: E402
from gpu_util import assert_same, dev, log, make_fill, oracle_many, pad_stride  # noqa: E402
from test_gpu_parity import DEFAULT, params  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = daq.Context(0)
    yield c
    c.set_schedule(*DEFAULT)
    c.close()


def _q_ref(x, N, Np, acc0):
    acc = acc0.copy()
    ped, Q = oracle.qmethod(x, N, ped_samples=Np, acc=acc)
    return ped, Q, acc


def _check_q(q, Q, acc, N, what):
    np.testing.assert_array_equal(q.qsum.cpu().numpy()[:len(Q)], Q, err_msg=what + ": qsum")
    a = q.acc.cpu().numpy()
    np.testing.assert_array_equal(a[:, :N], acc[:, :N], err_msg=what + ": acc")


@pytest.mark.parametrize("sched", [(256, 16, daq.DAQ_VARIANT_SPLIT, 0), (512, 8, daq.DAQ_VARIANT_SPLIT, 0),
                                   (256, 16, daq.DAQ_VARIANT_SPLIT, 3), (256, 16, daq.DAQ_VARIANT_RELOAD, 0)],
                         ids=["split256", "split512", "split_three_groups", "context_on_reload"])
def test_random_fills(ctx, sched):
    ctx.set_schedule(*sched)
    rng = np.random.default_rng(sched[0] + sched[2])
    shapes = [(1, 1), (3, 7), (54, 8), (54, 33), (2, 2047), (54, 2048), (5, 2049), (54, 4097), (7, 40_000),
              (54, 100_003), (54, 0)]
    fills, outs, qouts, refs = [], [], [], []
    for i, (C, N) in enumerate(shapes):
        x = rng.integers(1500, 2100, size=(C, max(N, 1))).astype(np.int16)
        # a few pulses so that islands exist
        for t in rng.integers(0, max(N, 1), size=max(N // 400, 1)):
            x[:, t:t + 6] -= rng.integers(20, 300, size=(C, 1)).astype(np.int16)
        x = pad_stride(x[:, :max(N, 1)])
        post = 700 if i == 8 else int(rng.integers(0, 40))  # one wide window (halo groups apart)
        p = params(-40 * C, int(rng.integers(0, 12)), post, int(rng.integers(1, 150)))
        f = make_fill(dev(x), N, p)
        o = daq.alloc_out(f)
        q = daq.alloc_q_out(f)
        q.ped = None  # the pedestals go to the T-method's output
        acc0 = rng.integers(-10_000, 10_000, size=q.acc.shape).astype(np.int32)
        q.acc.copy_(torch.from_numpy(acc0))
        fills.append(f)
        outs.append(o)
        qouts.append(q)
        refs.append((x, N, p, acc0))
    log("fused T+Q sched=%s" % (sched,))
    ctx.daq_process_batch_q(fills, outs, qouts)
    torch.cuda.synchronize()
    for i, (o, q, (x, N, p, acc0)) in enumerate(zip(outs, qouts, refs)):
        what = "fill %d C=%d N=%d" % (i, x.shape[0], N)
        ref = oracle.chop(x, n_samples=N, ped_samples=p["ped_samples"], threshold=p["threshold"], pre=p["pre"],
                          post=p["post"])
        assert_same(o, ref, ctx=what)
        ped, Q, acc = _q_ref(x, N, p["ped_samples"], acc0)
        np.testing.assert_array_equal(ped, ref.ped)
        _check_q(q, Q, acc, N, what)
    ctx.set_schedule(*DEFAULT)


def test_pedestals_to_the_q_output_and_argument_errors(ctx):
    rng = np.random.default_rng(5)
    x = pad_stride(rng.integers(1000, 3000, size=(54, 3001)).astype(np.int16))
    p = params(-200, 8, 24, 100)
    f = make_fill(dev(x), 3001, p)
    o = daq.alloc_out(f)
    o.ped = None
    q = daq.alloc_q_out(f)
    ctx.daq_process_batch_q([f], [o], [q])
    torch.cuda.synchronize()
    ref = oracle.chop(x, n_samples=3001, ped_samples=100, threshold=-200, pre=8, post=24)
    np.testing.assert_array_equal(q.ped.cpu().numpy(), ref.ped)
    ped, Q, acc = _q_ref(x, 3001, 100, np.zeros(q.acc.shape, np.int32))
    _check_q(q, Q, acc, 3001, "ped to q")
    o2 = daq.alloc_out(f)  # both pedestal outputs set
    with pytest.raises(daq.DaqError):
        ctx.daq_process_batch_q([f], [o2], [daq.alloc_q_out(f)])
    q3 = daq.alloc_q_out(f)
    with pytest.raises(daq.DaqError):  # two fills adding into one accumulator
        ctx.daq_process_batch_q([f, f], [daq.alloc_out(f), daq.alloc_out(f)],
                                [daq.QOut(q3.qsum, q3.acc, None), daq.QOut(None, q3.acc, None)])
    lib = daq.load_library()
    assert lib.daq_process_batch_q(ctx.handle, None, None, None, 0, None) == daq.DAQ_OK


def test_workload_16_fills_fused_and_separate(ctx):
    """The 16 benchmark fills: the fused call against the oracle, and against
    daq_process_batch followed by daq_qmethod_batch, element by element."""
    specs = synth.config_c1()
    xs = synth.render_many(specs)
    ns = [s.n_samples for s in specs]
    ps = [params(s.threshold, s.pre, s.post, s.ped_samples) for s in specs]
    refs = oracle_many(xs, ns, ps)
    fills = [make_fill(d, n, p) for d, n, p in zip(synth.to_device(xs), ns, ps)]
    outs = [daq.alloc_out(f) for f in fills]
    qouts = [daq.alloc_q_out(f) for f in fills]
    for q in qouts:
        q.ped = None
    log("fused T+Q on the 16 fills")
    ctx.daq_process_batch_q(fills, outs, qouts)
    torch.cuda.synchronize()
    for i, (o, r) in enumerate(zip(outs, refs)):
        assert_same(o, r, ctx="fill %d" % i)
    N = ns[0]
    ped, Q = oracle.qmethod(xs[0], N, ped_samples=ps[0]["ped_samples"])
    want = (xs[0][:, :N].astype(np.int64) - ped[:, None].astype(np.int64)).astype(np.int32)
    _check_q(qouts[0], Q, want, N, "fill 0")
    # the two separate calls give the same bytes
    outs2 = [daq.alloc_out(f) for f in fills]
    qouts2 = [daq.alloc_q_out(f) for f in fills]
    ctx.daq_process_batch(fills, outs2)
    ctx.daq_qmethod_batch(fills, qouts2)
    torch.cuda.synchronize()
    for i in range(len(fills)):
        assert torch.equal(qouts[i].qsum, qouts2[i].qsum), i
        assert torch.equal(qouts[i].acc, qouts2[i].acc), i
        assert torch.equal(outs[i].counts, outs2[i].counts), i


def test_capacity_overflow_leaves_the_q_method_exact(ctx):
    """Too small an island table: the T-method reports DAQ_STATUS_CAPACITY and
    keeps the records that fit; the Q-method outputs are unaffected."""
    x = np.full((54, 20_000), 1000, np.int16)
    x[0, 100:20_000:200] -= 500
    p = params(-100, 8, 24, 50)
    ref = oracle.chop(x, n_samples=20_000, ped_samples=50, threshold=-100, pre=8, post=24)
    assert ref.n_islands == 100
    f = make_fill(dev(x), 20_000, p)
    o = daq.alloc_out(f, capacity=37)
    q = daq.alloc_q_out(f)
    q.ped = None
    ctx.daq_process_batch_q([f], [o], [q])
    torch.cuda.synchronize()
    isl, n, total, status, ped, out = o.host()
    assert n == 100 and total == ref.total_len
    assert status & daq.DAQ_STATUS_CAPACITY
    np.testing.assert_array_equal(isl, ref.islands[:37])
    pq, Q, acc = _q_ref(x, 20_000, 50, np.zeros(q.acc.shape, np.int32))
    _check_q(q, Q, acc, 20_000, "capacity overflow")
