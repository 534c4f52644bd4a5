"""GPU tests of the serving loop (daq_server_* through the C ABI).

Each fill's results must be the same whether it is served alone or in a mix
of other fills arriving while batches run, and equal to the CPU oracle
(bit-exact: all integers). Admission follows the arena budget.
"""
import time

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU machines
    pytest.skip("no GPU", allow_module_level=True)

import paper_1611_04959_amd as daq  # noqa: E402
from gpu_util import log, oracle_many, poison, poison_slot  # noqa: E402


def _specs(n, seed):
    """Uneven small fills: lengths, rates, thresholds and windows vary."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        out.append(synth.FillSpec(seed=synth.fill_seed("serve-test", seed, i),
                                  n_samples=int(rng.integers(20_000, 90_001)),
                                  rate=float(rng.uniform(0.5, 4.0)),
                                  threshold=int(rng.integers(-400, -149)),
                                  pre=int(rng.integers(4, 17)), post=int(rng.integers(16, 49))))
    return out


@pytest.fixture(scope="module")
def workload():
    specs = _specs(12, 7)
    xs = synth.render_many(specs)
    refs = oracle_many(xs, [s.n_samples for s in specs],
                       [{"threshold": s.threshold, "pre": s.pre, "post": s.post, "ped_samples": s.ped_samples}
                        for s in specs])
    xd = synth.to_device(xs)
    fills = [daq.Fill(d, s.n_samples, threshold=s.threshold, pre=s.pre, post=s.post,
                      ped_samples=s.ped_samples) for d, s in zip(xd, specs)]
    return specs, xs, xd, fills, refs


@pytest.fixture(scope="module")
def ctx():
    c = daq.Context(0)
    c.set_schedule(256, 16, daq.DAQ_VARIANT_SPLIT)
    yield c
    c.close()


def _drain(srv, want, timeout_s=60.0):
    got = {}
    t_end = time.time() + timeout_s
    while len(got) < want:
        assert time.time() < t_end, "server did not finish"
        for c in srv.poll(64, 20_000):
            got[c.ticket] = c
    return got


def _check(srv, c, ref, C, what):
    assert c.error == daq.DAQ_OK, what
    assert c.status == 0, what
    assert c.n_islands == ref.n_islands and c.total_len == ref.total_len, what
    isl, ped, out = srv.results(c, C)
    np.testing.assert_array_equal(isl, ref.islands, err_msg=what + ": islands")
    np.testing.assert_array_equal(ped, ref.ped, err_msg=what + ": ped")
    np.testing.assert_array_equal(out, ref.out, err_msg=what + ": out")
    poison_slot(srv, c, C)  # the slot's next user starts from poison
    return isl, ped, out


def test_alone_equals_in_the_mix(ctx, workload):
    specs, xs, xd, fills, refs = workload
    C = synth.CHANNELS
    need = max(daq.slot_bytes(f) for f in fills)
    arena = poison(torch.empty(6 * need, dtype=torch.uint8, device="cuda"))  # room for ~6 fills at once
    with daq.Server(ctx, arena, n_streams=3, max_batch=4) as srv:
        alone = {}
        for i, f in enumerate(fills):
            log("server alone fill %d N=%d" % (i, specs[i].n_samples))
            t = srv.submit(f, tag=i)
            assert t is not None
            (c,) = _drain(srv, 1).values()
            assert c.tag == i and c.batch_fills == 1
            alone[i] = _check(srv, c, refs[i], C, "alone %d" % i)
            srv.release(t)
        # the mix: everything at once, admitted as the budget frees up
        log("server mix of %d fills" % len(fills))
        order = list(range(len(fills))) * 2
        pending, got, rejected = list(order), [], 0
        t_end = time.time() + 60
        while pending or len(got) < len(order):
            assert time.time() < t_end, "mix did not finish"
            while pending:
                t = srv.submit(fills[pending[0]], tag=pending[0])
                if t is None:
                    rejected += 1
                    break
                pending.pop(0)
            for c in srv.poll(64, 2_000):
                i = c.tag
                isl, ped, out = _check(srv, c, refs[i], C, "mix %d" % i)
                np.testing.assert_array_equal(isl, alone[i][0])
                np.testing.assert_array_equal(out, alone[i][2])
                got.append(c)
                srv.release(c.ticket)
        st = srv.stats()
        log("mix: %d batches, %d rejected submits, peak %.1f MB of %.1f MB" %
            (st.batches, st.rejected, st.arena_peak / 1e6, st.arena_bytes / 1e6))
        assert rejected > 0 and st.rejected == rejected  # the budget did bind
        assert st.arena_peak <= st.arena_bytes
        assert st.pending == 0 and st.running == 0 and st.arena_in_use == 0
        assert max(c.batch_fills for c in got) > 1  # fills were batched


def test_batches_overlap_on_the_device(ctx, workload):
    specs, xs, xd, fills, refs = workload
    need = sum(daq.slot_bytes(f) for f in fills)
    arena = poison(torch.empty(need + (1 << 20), dtype=torch.uint8, device="cuda"))
    with daq.Server(ctx, arena, n_streams=3, max_batch=2) as srv:
        for rep in range(3):
            tickets = [srv.submit(f, tag=i) for i, f in enumerate(fills)]
            assert all(t is not None for t in tickets)
            got = _drain(srv, len(fills))
            spans = sorted((c.t_launch_ns, c.t_ready_ns) for c in got.values())
            overlap = any(b0 < a1 for (a0, a1), (b0, b1) in zip(spans, spans[1:]))
            for c in got.values():
                _check(srv, c, refs[c.tag], synth.CHANNELS, "overlap %d" % c.tag)
                assert c.t_submit_ns <= c.t_launch_ns <= c.t_ready_ns
                srv.release(c.ticket)
            if overlap:
                break
        assert overlap, "no two batches were in flight together"


def test_host_fed_fills_match(ctx, workload):
    specs, xs, xd, fills, refs = workload
    host = [torch.from_numpy(x).pin_memory() for x in xs[:3]]
    need = sum(daq.slot_bytes(f, host_raw=True) for f in fills[:3])
    arena = poison(torch.empty(need, dtype=torch.uint8, device="cuda"))
    with daq.Server(ctx, arena, n_streams=2, max_batch=2) as srv:
        for i in range(3):
            assert srv.submit(fills[i], tag=i, host_raw=host[i]) is not None
        got = _drain(srv, 3)
        for c in got.values():
            _check(srv, c, refs[c.tag], synth.CHANNELS, "host-fed %d" % c.tag)
            srv.release(c.ticket)


def test_host_packed12_fills_match(ctx, workload):
    """Fills submitted as 12-bit words: copied, unpacked on the device, chopped."""
    specs, xs, xd, fills, refs = workload
    if min(int(x.min()) for x in xs[:3]) < 0 or max(int(x.max()) for x in xs[:3]) > 4095:
        pytest.skip("test fills are not 12-bit")
    host = []
    for x, s in zip(xs[:3], specs[:3]):
        N = s.n_samples
        pst = daq.packed12_stride(N)
        v = x[:, :N].astype(np.uint32) & 0xFFF
        if N % 2:
            v = np.concatenate([v, np.zeros((v.shape[0], 1), np.uint32)], axis=1)
        a, b = v[:, 0::2], v[:, 1::2]
        trip = np.stack([a & 0xFF, (a >> 8) | ((b & 0xF) << 4), b >> 4], axis=2).reshape(v.shape[0], -1)
        p = np.zeros((x.shape[0], pst), np.uint8)
        nb = (3 * N + 1) // 2
        p[:, :nb] = trip[:, :nb]
        host.append(torch.from_numpy(p).pin_memory())
    need = sum(daq.slot_bytes(f, host_packed12=True) for f in fills[:3])
    arena = poison(torch.empty(need, dtype=torch.uint8, device="cuda"))
    with daq.Server(ctx, arena, n_streams=2, max_batch=2) as srv:
        for i in range(3):
            assert srv.submit(fills[i], tag=i, host_packed12=host[i]) is not None
        got = _drain(srv, 3)
        for c in got.values():
            _check(srv, c, refs[c.tag], synth.CHANNELS, "host-packed %d" % c.tag)
            srv.release(c.ticket)


def test_admission_and_release_rules(ctx, workload):
    specs, xs, xd, fills, refs = workload
    f = fills[0]
    one = daq.slot_bytes(f)
    arena = poison(torch.empty(2 * one + 1024, dtype=torch.uint8, device="cuda"))
    with daq.Server(ctx, arena, n_streams=1, max_batch=8) as srv:
        t1 = srv.submit(f, tag=1)
        t2 = srv.submit(f, tag=2)
        assert t1 is not None and t2 is not None
        assert srv.submit(f, tag=3) is None          # budget full: DAQ_EAGAIN
        big = daq.Fill(xd[0], specs[0].n_samples, threshold=f.threshold, pre=f.pre, post=f.post)
        with pytest.raises(daq.DaqError) as e:        # a slot that can never fit
            srv.submit(daq.Fill(torch.empty((54, 8 * (arena.numel() // 54 // 16 + 8)), dtype=torch.int16,
                                            device="cuda"), 8 * (arena.numel() // 54 // 16 + 8)))
        assert e.value.code == daq.DAQ_ERANGE
        got = _drain(srv, 2)
        assert sorted(c.tag for c in got.values()) == [1, 2]
        srv.release(t1)
        assert srv.try_release(t1) == daq.DAQ_EINVAL  # already released
        assert srv.try_release(12345) == daq.DAQ_EINVAL
        t3 = srv.submit(big, tag=3)
        assert t3 is not None
        _drain(srv, 1)
        srv.release(t2)
        srv.release(t3)
        assert srv.stats().arena_in_use == 0


def test_persistent_schedule_serves_the_same(workload):
    """Workers inherit the context's schedule: the persistent kernel behind the server."""
    specs, xs, xd, fills, refs = workload
    C = synth.CHANNELS
    c2 = daq.Context(0)
    try:
        c2.set_schedule(512, 2, daq.DAQ_VARIANT_PIPE)
        need = sum(daq.slot_bytes(f) for f in fills)
        arena = poison(torch.empty(need, dtype=torch.uint8, device="cuda"))
        with daq.Server(c2, arena, n_streams=2, max_batch=4) as srv:
            log("server with the persistent schedule: %d fills" % len(fills))
            for i, f in enumerate(fills):
                assert srv.submit(f, tag=i) is not None
            got = _drain(srv, len(fills))
            for c in got.values():
                _check(srv, c, refs[c.tag], C, "persistent %d" % c.tag)
                srv.release(c.ticket)
    finally:
        c2.close()


def test_serving_burst_full_size(ctx):
    """Serving-configuration fills at their own shape (54 x 560,000, the
    streams' nominal distributions): each fill served alone, then a burst of
    ten submitted at once to a server whose budget holds three slots, so
    admission refuses fills until slots are released. Every completion equals
    the oracle and the same fill served alone; the arena and every released
    slot hold poison."""
    specs = [synth.config_c3_fill(s, 0) for s in range(10)]
    xs = synth.render_many(specs)
    log("serving burst: oracle on %d full-size fills" % len(specs))
    refs = oracle_many(xs, [s.n_samples for s in specs],
                       [{"threshold": s.threshold, "pre": s.pre, "post": s.post, "ped_samples": s.ped_samples}
                        for s in specs])
    xd = synth.to_device(xs)
    fills = [daq.Fill(d, s.n_samples, threshold=s.threshold, pre=s.pre, post=s.post,
                      ped_samples=s.ped_samples) for d, s in zip(xd, specs)]
    C = synth.CHANNELS
    need = max(daq.slot_bytes(f) for f in fills)
    arena = poison(torch.empty(3 * need + 4096, dtype=torch.uint8, device="cuda"))
    with daq.Server(ctx, arena, n_streams=3, max_batch=16) as srv:
        alone = {}
        for i, f in enumerate(fills):
            log("serving burst: fill %d alone" % i)
            t = srv.submit(f, tag=i)
            assert t is not None
            (c,) = _drain(srv, 1).values()
            assert c.tag == i and c.batch_fills == 1
            alone[i] = _check(srv, c, refs[i], C, "alone %d" % i)
            srv.release(t)
        log("serving burst: %d fills at once, budget of 3 slots" % len(fills))
        pending, got, rejected = list(range(len(fills))), [], 0
        t_end = time.time() + 120
        while pending or len(got) < len(fills):
            assert time.time() < t_end, "burst did not finish"
            while pending:
                t = srv.submit(fills[pending[0]], tag=pending[0])
                if t is None:
                    rejected += 1
                    break
                pending.pop(0)
            for c in srv.poll(64, 2_000):
                i = c.tag
                isl, ped, out = _check(srv, c, refs[i], C, "burst %d" % i)
                np.testing.assert_array_equal(isl, alone[i][0])
                np.testing.assert_array_equal(ped, alone[i][1])
                np.testing.assert_array_equal(out, alone[i][2])
                got.append(c)
                srv.release(c.ticket)
        st = srv.stats()
        log("serving burst: %d batches, %d refused submits, largest batch %d" %
            (st.batches, rejected, max(c.batch_fills for c in got)))
        assert rejected > 0 and st.rejected == rejected  # the budget did bind
        assert sorted(c.tag for c in got) == list(range(len(fills)))
        assert st.arena_in_use == 0


def test_deadtime_accounting_and_watchdog(ctx, workload):
    """Forced from the host, every kernel running normally: a fill whose
    arrival lies 50 ms back is late against the 10 ms admission deadline; the
    time between a refused submit and the next admission is deadtime; a 1 us
    batch time-out makes the watchdog give up on batches that are still
    running (their fills complete with DAQ_ETIMEDOUT and their slots are held
    until the device is done with them); with the time-out back at 10 s the
    server serves exact results again."""
    specs, xs, xd, fills, refs = workload
    C = synth.CHANNELS
    size = [daq.slot_bytes(f) for f in fills]
    order = sorted(range(len(fills)), key=lambda i: size[i])
    small, big1, big2 = order[0], order[-1], order[-2]
    arena = poison(torch.empty(size[big1] + size[big2] + 256, dtype=torch.uint8, device="cuda"))
    with daq.Server(ctx, arena, n_streams=2, max_batch=2) as srv:
        srv.set_limits(admit_deadline_us=10_000, batch_timeout_us=10_000_000)
        # late admission
        t_arr = time.monotonic_ns() - 50_000_000
        t = srv.submit(fills[small], tag=small, arrival_ns=t_arr)
        (c,) = _drain(srv, 1).values()
        _check(srv, c, refs[small], C, "late fill")
        assert c.t_submit_ns == t_arr and c.t_ready_ns - c.t_submit_ns >= 50_000_000
        st = srv.stats()
        assert st.late == 1 and st.admit_wait_max_ns >= 50_000_000 and st.deadtime_ns == 0
        srv.release(t)
        # deadtime: the budget holds the two largest fills; a third is refused
        t1 = srv.submit(fills[big1], tag=big1)
        t2 = srv.submit(fills[big2], tag=big2)
        assert t1 is not None and t2 is not None
        assert srv.submit(fills[small], tag=small) is None
        time.sleep(0.02)
        for c in _drain(srv, 2).values():
            _check(srv, c, refs[c.tag], C, "deadtime %d" % c.tag)
        srv.release(t1)
        srv.release(t2)
        t3 = srv.submit(fills[small], tag=small)
        assert t3 is not None
        st = srv.stats()
        assert st.deadtime_ns >= 20_000_000 and st.rejected == 1
        _drain(srv, 1)
        srv.release(t3)
        # watchdog: a 1 us time-out expires while the batches still run
        srv.set_limits(admit_deadline_us=10_000, batch_timeout_us=1)
        tickets = [srv.submit(fills[i], tag=i) for i in (big1, big2)]
        assert all(t is not None for t in tickets)
        got = _drain(srv, 2)
        timed_out = [c for c in got.values() if c.error == daq.DAQ_ETIMEDOUT]
        assert timed_out, "no batch outlived a 1 us time-out"
        for c in got.values():
            assert c.error in (daq.DAQ_OK, daq.DAQ_ETIMEDOUT)
            if c.error == daq.DAQ_ETIMEDOUT:
                assert c.n_islands == 0 and c.total_len == 0
            srv.release(c.ticket)
        assert srv.stats().timed_out == len(timed_out)
        t_end = time.time() + 10
        while srv.stats().arena_in_use != 0:  # held slots come back once the device is done
            assert time.time() < t_end, "held slots were not reclaimed"
            time.sleep(0.005)
        # and back to normal
        srv.set_limits(admit_deadline_us=10_000, batch_timeout_us=10_000_000)
        t4 = srv.submit(fills[big1], tag=big1)
        (c,) = _drain(srv, 1).values()
        _check(srv, c, refs[big1], C, "after the watchdog")
        srv.release(t4)
        with pytest.raises(daq.DaqError):
            srv.set_limits(admit_deadline_us=-1)


def test_consumer_that_never_polls_loses_nothing(ctx, workload):
    """A consumer that stops polling and releasing: the budget fills, every
    later submit is refused with DAQ_EAGAIN (none is admitted and dropped),
    the refusals count as deadtime, and when the consumer comes back every
    admitted fill's completion is there, exact."""
    specs, xs, xd, fills, refs = workload
    C = synth.CHANNELS
    size = [daq.slot_bytes(f) for f in fills]
    budget = sum(sorted(size)[:4]) + 256
    arena = poison(torch.empty(budget, dtype=torch.uint8, device="cuda"))
    with daq.Server(ctx, arena, n_streams=2, max_batch=4) as srv:
        admitted, refused = {}, 0
        t_end = time.time() + 0.3
        k = 0
        while time.time() < t_end:  # submit round-robin, never poll
            i = k % len(fills)
            k += 1
            t = srv.submit(fills[i], tag=i)
            if t is None:
                refused += 1
            else:
                admitted[t] = i
        log("never-polling consumer: %d admitted, %d refused" % (len(admitted), refused))
        assert len(admitted) >= 1 and refused > 100
        st = srv.stats()
        assert st.submitted == len(admitted) and st.rejected == refused
        assert st.arena_in_use <= budget
        time.sleep(0.05)
        got = _drain(srv, len(admitted))
        assert sorted(got) == sorted(admitted)
        for t, c in got.items():
            assert c.tag == admitted[t]
            _check(srv, c, refs[c.tag], C, "never-polled %d" % c.tag)
            srv.release(t)
        assert srv.submit(fills[0], tag=0) is not None  # admits again, and the dead period ends
        st = srv.stats()
        assert st.deadtime_ns > 0 and st.completed == len(admitted)
        _drain(srv, 1)
