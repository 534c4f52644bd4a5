"""GPU parity on fills laid out the way a caller's buffers may be: rows
further apart than N (row_stride well above the row's samples), a raw base
inside a larger allocation (16-byte aligned, not 256), and every byte
outside the fill's rows (before the base, between rows, after the last row)
filled with random int16 values over the whole range. Each case is compared
with the oracle element by element for every schedule family and all three
entry forms, and for the Q-method and both methods on one read, so a kernel
that reads a sample outside [0, N) of a row, or relies on an alignment the
header does not promise, fails."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU machines
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_1611_04959_amd as daq  # noqa: E402
from gpu_util import assert_same, log, oracle_result, poison, run  # noqa: E402

# (C, N, row_stride, base offset in elements, threshold, pre, post, Np)
CASES = [
    (54, 20_003, 20_072, 8, -200, 8, 24, 100),
    (5, 4_049, 4_064, 24, -150, 4, 16, 100),
    (1, 8, 8, 0, -100, 0, 0, 1),
    (54, 12_000, 16_096, 4_096, -300, 15, 31, 100),
    (17, 100, 104, 56, -100, 3, 5, 100),
    (54, 99, 200, 8, -200, 8, 24, 100),
    (3, 70_001, 70_016, 16, -120, 2, 40, 37),
]
# one schedule of each family: split (one group, fill groups), reload,
# registers, LDS, persistent
SCHEDULES = [(512, 8, 5, 0), (256, 16, 5, 2), (256, 4, 0, 0), (256, 1, 1, 0), (256, 2, 2, 0), (256, 4, 6, 0)]
MODES = ["chop", "twopass", "batch"]


def _case(rng, C, N, S, off):
    """Host rows with pulses, and a device buffer holding them at `off` with
    row stride S, everything else random."""
    x = (1800 + rng.integers(-3, 4, (C, N))).astype(np.int16)
    for t0 in rng.integers(0, max(N - 30, 1), max(N // 700, 2)):
        c0 = int(rng.integers(0, C))
        x[c0:c0 + 2, t0:t0 + 20] -= int(rng.integers(150, 900))
    tail = int(rng.integers(0, 300))
    buf = rng.integers(-32768, 32768, off + C * S + tail).astype(np.int16)
    for c in range(C):
        buf[off + c * S:off + c * S + N] = x[c]
    d = torch.from_numpy(buf).to("cuda")
    raw = d.as_strided((C, max(daq.padded(N), 8)), (S, 1), off)
    host = np.stack([buf[off + c * S:off + c * S + S] for c in range(C)])
    return raw, host, d


@pytest.fixture(scope="module")
def ctx():
    c = daq.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def cases():
    rng = np.random.default_rng(2024)
    out = []
    for (C, N, S, off, thr, pre, post, np_) in CASES:
        raw, host, keep = _case(rng, C, N, S, off)
        p = {"threshold": thr, "pre": pre, "post": post, "ped_samples": np_}
        out.append((raw, host, keep, N, p, oracle_result(host, N, p)))
    return out


@pytest.mark.parametrize("sched", SCHEDULES, ids=lambda s: "t%d_w%d_v%d_p%d" % s)
def test_strided_offset_fills_with_junk_around_them(ctx, cases, sched):
    ctx.set_schedule(*sched)
    assert any(r.n_islands > 0 for *_, r in cases)
    for mode in MODES:
        log("layouts sched=%s mode=%s" % (sched, mode))
        fills = [daq.Fill(raw, N, threshold=p["threshold"], pre=p["pre"], post=p["post"],
                          ped_samples=p["ped_samples"]) for raw, _, _, N, p, _ in cases]
        outs = [daq.alloc_out(f) for f in fills]
        run(ctx, mode, fills, outs)
        for i, (o, (*_, ref)) in enumerate(zip(outs, cases)):
            assert_same(o, ref, ctx="case %d %s sched %s" % (i, mode, sched))
    ctx.set_schedule(512, 8, 5, 0)


def _q_refs(cases, rng):
    """Oracle Q-method of every case (pedestals, decimated sums, accumulator
    rows after adding into random starting values) and those starting values."""
    out = []
    for raw, host, _, N, p, _ in cases:
        acc0 = rng.integers(-10_000, 10_000, size=(raw.shape[0], raw.shape[1])).astype(np.int32)
        acc = acc0.copy()
        ped, Q = oracle.qmethod(host, N, ped_samples=p["ped_samples"], acc=acc)
        out.append((acc0, ped, Q, acc))
    return out


def _q_outs(fills, qrefs, with_ped=True):
    qs = []
    for f, (acc0, *_) in zip(fills, qrefs):
        q = daq.alloc_q_out(f)
        poison(q.qsum)
        if with_ped:
            poison(q.ped)
        else:
            q.ped = None
        q.acc.copy_(torch.from_numpy(acc0))
        qs.append(q)
    return qs


def _check_q(q, qref, N, what):
    acc0, ped, Q, acc = qref
    if q.ped is not None:
        np.testing.assert_array_equal(q.ped.cpu().numpy(), ped, err_msg=what + ": ped")
    np.testing.assert_array_equal(q.qsum.cpu().numpy()[:len(Q)], Q, err_msg=what + ": qsum")
    a = q.acc.cpu().numpy()
    np.testing.assert_array_equal(a[:, :N], acc[:, :N], err_msg=what + ": acc")
    np.testing.assert_array_equal(a[:, N:], acc0[:, N:], err_msg=what + ": acc past N")


@pytest.mark.parametrize("threads", [256, 512])
def test_qmethod_on_strided_offset_fills(ctx, cases, threads):
    ctx.set_schedule(threads, 8, daq.DAQ_VARIANT_SPLIT)
    qrefs = _q_refs(cases, np.random.default_rng(threads))
    fills = [daq.Fill(raw, N, ped_samples=p["ped_samples"]) for raw, _, _, N, p, _ in cases]
    for mode in ("single", "batch"):
        log("layouts q-method threads=%d mode=%s" % (threads, mode))
        qs = _q_outs(fills, qrefs)
        if mode == "single":
            for f, q in zip(fills, qs):
                ctx.daq_qmethod_batch([f], [q])
        else:
            ctx.daq_qmethod_batch(fills, qs)
        torch.cuda.synchronize()
        for i, (q, qref, case) in enumerate(zip(qs, qrefs, cases)):
            _check_q(q, qref, case[3], "case %d q %s" % (i, mode))
    ctx.set_schedule(512, 8, 5, 0)


@pytest.mark.parametrize("sched", [(512, 8, 5, 0), (256, 16, 5, 3)], ids=["split512", "split_three_groups"])
def test_both_methods_on_strided_offset_fills(ctx, cases, sched):
    ctx.set_schedule(*sched)
    qrefs = _q_refs(cases, np.random.default_rng(sched[1]))
    fills = [daq.Fill(raw, N, threshold=p["threshold"], pre=p["pre"], post=p["post"],
                      ped_samples=p["ped_samples"]) for raw, _, _, N, p, _ in cases]
    outs = [daq.alloc_out(f) for f in fills]
    qs = _q_outs(fills, qrefs, with_ped=False)  # the pedestals go to the T-method's output
    log("layouts fused T+Q sched=%s" % (sched,))
    ctx.daq_process_batch_q(fills, outs, qs)
    torch.cuda.synchronize()
    for i, (o, q, qref, case) in enumerate(zip(outs, qs, qrefs, cases)):
        assert_same(o, case[5], ctx="case %d fused T" % i)
        _check_q(q, qref, case[3], "case %d fused Q" % i)
    ctx.set_schedule(512, 8, 5, 0)
