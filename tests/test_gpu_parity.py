"""GPU parity: the HIP library (through its C ABI) against the CPU oracle,
element by element, bit-exact (every quantity is an integer).

Covers hand-derived fixtures, random small fills spanning several tiles with
ragged tails, every schedule, the three entry forms (fused per fill, find +
gather, batched launch), edge cases, and the benchmark workloads at full size.
"""
import ctypes
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU machines
    pytest.skip("no GPU", allow_module_level=True)

import golden_io  # noqa: E402
import paper_1611_04959_amd as daq  # noqa: E402
from gpu_util import (assert_same, dev, log, make_fill, oracle_many, oracle_result, pad_stride,  # noqa: E402
                      poison, poison_out, run)

SCHEDULES = [(256, 2, 2, 0), (256, 1, 2, 0), (256, 0, 2, 0), (256, 4, 0, 0), (256, 1, 1, 0), (512, 2, 0, 0),
             (512, 1, 1, 0), (128, 8, 0, 0), (128, 2, 1, 0), (256, 0, 0, 0), (512, 0, 1, 0), (256, 4, 3, 0),
             (512, 2, 3, 0), (256, 3, 4, 0), (256, 8, 5, 0), (512, 2, 5, 0), (256, 0, 5, 0), (256, 16, 5, 2),
             (256, 16, 5, 3), (512, 4, 5, 4), (256, 0, 5, 2), (256, 4, 6, 0), (512, 2, 6, 0), (256, 0, 6, 0),
             (256, 1, 6, 0), (512, 8, 5, 0)]
MODES = ["chop", "twopass", "batch"]
DEFAULT = (512, 8, 5, 0)  # the library's default schedule


@pytest.fixture(scope="module")
def ctx():
    c = daq.Context(0)
    yield c
    c.close()


def params(thr, pre, post, np_=100):
    return {"threshold": thr, "pre": pre, "post": post, "ped_samples": np_}


@pytest.mark.parametrize("path", golden_io.fixture_files(), ids=lambda p: p.split("/")[-1])
@pytest.mark.parametrize("mode", MODES)
def test_golden_fixtures(ctx, path, mode):
    g = golden_io.load(path)
    log("golden %s mode=%s" % (path.split("/")[-1], mode))
    x = pad_stride(g["x"])
    p = params(g["threshold"], g["pre"], g["post"], g["ped_samples"])
    f = make_fill(dev(x), g["samples"], p)
    o = daq.alloc_out(f)
    run(ctx, mode, [f], [o])
    ref = oracle_result(x, g["samples"], p)
    assert_same(o, ref, ctx=g["name"])
    # and the hand-derived values themselves
    isl, n, total, status, ped, out = o.host()
    np.testing.assert_array_equal(isl, g["islands"])
    np.testing.assert_array_equal(out, g["out"])


def _random_fill(rng, C, N):
    """Pulse-like fill with dense and sparse regions and extreme values."""
    x = rng.integers(995, 1006, size=(C, N)).astype(np.int16)
    n_p = int(rng.integers(0, max(2, N // 40)))
    for _ in range(n_p):
        t = int(rng.integers(0, N))
        L = int(rng.integers(1, 30))
        x[rng.integers(0, C), t:t + L] -= np.int16(rng.integers(0, 400))
    if rng.random() < 0.3:   # a dense block that makes a long island
        a = int(rng.integers(0, N))
        x[:, a:a + int(rng.integers(100, 3000))] -= 300
    return pad_stride(x)


@pytest.mark.parametrize("sched", SCHEDULES, ids=lambda s: "t%d_w%d_v%d_p%d" % s)
def test_random_fills_all_schedules_and_modes(ctx, sched):
    ctx.set_schedule(*sched)
    rng = np.random.default_rng(sum(sched) * 7919)
    shapes = [(54, 1), (54, 7), (54, 8), (54, 2047), (54, 2048), (54, 2049), (54, 4097),
              (54, 12_345), (54, 40_000), (1, 5000), (3, 9999), (7, 4100), (54, 0)]
    for C, N in shapes:
        x = _random_fill(rng, C, max(N, 1))[:, :max(daq.padded(N), 8)]
        for pre, post in ((8, 24), (0, 0), (1, 0), (40, 3), (300, 700)):
            Np = int(rng.integers(1, 150))
            S = x[:, :N].astype(np.int64).sum(0)
            thr = int(np.quantile(S, 0.1) - S[:min(N, Np)].mean()) if N > 0 else -5
            p = params(thr, pre, post, Np)
            ref = oracle_result(x, N, p)
            for mode in MODES:
                log("random C=%d N=%d pre=%d post=%d sched=%s mode=%s" % (C, N, pre, post, sched, mode))
                f = make_fill(dev(x), N, p)
                o = daq.alloc_out(f)
                run(ctx, mode, [f], [o])
                assert_same(o, ref, ctx="C=%d N=%d pre=%d post=%d %s %s" % (C, N, pre, post, sched, mode))
    ctx.set_schedule(*DEFAULT)


def test_batch_of_uneven_random_fills(ctx):
    rng = np.random.default_rng(5)
    xs, ns, ps = [], [], []
    for i in range(40):
        C = int(rng.choice([54, 54, 54, 1, 5]))
        N = int(rng.integers(0, 30_000))
        xs.append(_random_fill(rng, C, max(N, 1))[:, :max(daq.padded(N), 8)])
        ns.append(N)
        ps.append(params(int(rng.integers(-400, 0)), int(rng.integers(0, 20)), int(rng.integers(0, 60)),
                         int(rng.integers(1, 200))))
    refs = oracle_many(xs, ns, ps)
    for sched in SCHEDULES:
        ctx.set_schedule(*sched)
        log("uneven batch sched=%s" % (sched,))
        fills = [make_fill(dev(x), n, p) for x, n, p in zip(xs, ns, ps)]
        outs = [daq.alloc_out(f) for f in fills]
        run(ctx, "batch", fills, outs)
        for i, (o, r) in enumerate(zip(outs, refs)):
            assert_same(o, r, ctx="fill %d sched %s" % (i, sched))
    ctx.set_schedule(*DEFAULT)


@pytest.mark.parametrize("sched", [(256, 2, 2, 0), (256, 16, 5, 0), (256, 16, 5, 3), (256, 4, 6, 0)],
                         ids=lambda s: "t%d_w%d_v%d_p%d" % s)
def test_graph_replays_match_eager(ctx, sched):
    """Replays of the captured graphs, with eager work and syncs between them."""
    rng = np.random.default_rng(17 + sched[3])
    ctx.set_schedule(*sched)
    for rep in range(4):
        n = int(rng.integers(2, 9))
        xs = [_random_fill(rng, 54, int(rng.integers(1000, 20_000))) for _ in range(n)]
        ns = [x.shape[1] - int(rng.integers(0, 8)) for x in xs]
        ps = [params(-150, 8, 24) for _ in range(n)]
        refs = oracle_many(xs, ns, ps)
        fills = [make_fill(dev(x), nn, p) for x, nn, p in zip(xs, ns, ps)]
        for graphs in (True, False):
            ctx.set_graphs(graphs)
            outs = [daq.alloc_out(f) for f in fills]
            log("graph replay rep=%d graphs=%s n=%d" % (rep, graphs, n))
            run(ctx, "batch", fills, outs)
            torch.zeros(1000, device="cuda").add_(1)   # eager work between replays
            torch.cuda.synchronize()
            for o, r in zip(outs, refs):
                assert_same(o, r, ctx="rep %d graphs %s" % (rep, graphs))
    ctx.set_graphs(True)


def test_edge_cases(ctx):
    C = 54
    base = np.full((C, 4096), 1000, np.int16)
    cases = []
    cases.append(("empty fill", base[:, :8], 0, params(-10, 8, 24)))
    cases.append(("one sample", base[:, :8], 1, params(1, 8, 24)))
    cases.append(("all below", base, 4096, params(1, 8, 24)))
    cases.append(("no crossing", base, 4096, params(-1, 8, 24)))
    x = base.copy()
    x[0, 0] -= 500
    x[0, 4095] -= 500
    cases.append(("crossing at both ends", x, 4096, params(-100, 8, 24, 1000)))
    x = np.full((C, 100_000), 1000, np.int16)
    x[3, 50_000] -= 400
    cases.append(("widest windows", x, 100_000, params(-100, daq.DAQ_MAX_WINDOW, daq.DAQ_MAX_WINDOW)))
    x = np.full((C, 3000), 1000, np.int16)
    x[:, ::2] = -32768
    x[:, 1::2] = 32767
    cases.append(("int16 extremes", x, 3000, params(0, 2, 2, 1)))
    cases.append(("int16 extremes thr max", x, 3000, params(2**31 - 1, 0, 0, 2)))
    cases.append(("thr min", x, 3000, params(-2**31, 0, 0, 2)))
    x = np.full((C, 10_000), 1000, np.int16)
    x[7, 0:10_000:3] -= 300
    cases.append(("dense pre=post=0", x, 10_000, params(-100, 0, 0, 1)))
    cases.append(("touching windows", x, 10_000, params(-100, 1, 0, 1)))
    for name, x, N, p in cases:
        for mode in MODES:
            log("edge %s mode=%s" % (name, mode))
            f = make_fill(dev(x), N, p)
            o = daq.alloc_out(f)
            run(ctx, mode, [f], [o])
            assert_same(o, oracle_result(x, N, p), ctx=name + " " + mode)


def test_capacity_and_out_stride_overflow(ctx):
    x = np.full((54, 20_000), 1000, np.int16)
    x[0, 100:20_000:200] -= 500
    p = params(-100, 8, 24, 50)
    ref = oracle_result(x, 20_000, p)
    assert ref.n_islands == 100
    for mode in MODES:
        log("capacity overflow mode=%s" % mode)
        f = make_fill(dev(x), 20_000, p)
        o = daq.alloc_out(f, capacity=37)
        run(ctx, mode, [f], [o])
        isl, n, total, status, ped, out = o.host()
        assert n == 100 and total == ref.total_len
        assert status & daq.DAQ_STATUS_CAPACITY
        np.testing.assert_array_equal(isl, ref.islands[:37])
        k = int(ref.islands[36, 2] + ref.islands[36, 1] - ref.islands[36, 0])
        np.testing.assert_array_equal(out[:, :k], ref.out[:, :k])
    for mode in MODES:
        log("out stride overflow mode=%s" % mode)
        f = make_fill(dev(x), 20_000, p)
        o = daq.alloc_out(f)
        o.out = poison(torch.empty((54, 1000), dtype=torch.int16, device="cuda"))
        run(ctx, mode, [f], [o])
        isl, n, total, status, ped, out = o.host()
        assert status == daq.DAQ_STATUS_OUT_STRIDE and total == ref.total_len > 1000
        np.testing.assert_array_equal(isl, ref.islands)
        np.testing.assert_array_equal(out, ref.out[:, :1000])


def test_schedule_validation(ctx):
    bad = [(128, 4, daq.DAQ_VARIANT_PIPE, 0), (256, 4, daq.DAQ_VARIANT_PIPE, 2), (256, 17, 5, 0),
           (256, 4, 7, 0), (256, 4, daq.DAQ_VARIANT_SPLIT, 5), (512, 4, daq.DAQ_VARIANT_LDS, 0)]
    lib = daq.load_library()
    for sc in bad:
        s = daq.daq_schedule(*sc)
        assert lib.daq_ctx_set_schedule(ctx.handle, ctypes.byref(s)) == daq.DAQ_EINVAL, sc
    ctx.set_schedule(*DEFAULT)


def test_argument_errors(ctx):
    x = dev(np.zeros((54, 64), np.int16))
    good = daq.Fill(x, 64)
    o = daq.alloc_out(good)
    with pytest.raises(daq.DaqError):
        ctx.daq_chop_fill(daq.Fill(x, 65), o)               # N > row stride
    with pytest.raises(daq.DaqError):
        ctx.daq_chop_fill(daq.Fill(x, 64, pre=-1), o)
    with pytest.raises(daq.DaqError):
        ctx.daq_chop_fill(daq.Fill(x, 64, pre=daq.DAQ_MAX_WINDOW + 1), o)
    with pytest.raises(daq.DaqError):
        ctx.daq_chop_fill(daq.Fill(x, 64, ped_samples=0), o)
    odd = dev(np.zeros((54, 60), np.int16))
    with pytest.raises(daq.DaqError) as e:
        ctx.daq_chop_fill(daq.Fill(odd, 60), o)             # stride not a multiple of 8
    assert e.value.code == daq.DAQ_EALIGN
    with pytest.raises(daq.DaqError) as e:
        ctx.daq_chop_fill(daq.Fill(x[:, 1:], 63), o)          # base not 16-byte aligned
    assert e.value.code == daq.DAQ_EALIGN
    torch.cuda.synchronize()


def test_repeat_runs_identical(ctx):
    spec = synth.config_c1(1)[0]
    x = synth.render(spec)
    f = make_fill(dev(x), spec.n_samples, params(spec.threshold, spec.pre, spec.post))
    prev = None
    for i in range(3):
        o = daq.alloc_out(f)
        run(ctx, "chop", [f], [o])
        cur = o.host()
        if prev is not None:
            for a, b in zip(prev, cur):
                if isinstance(a, np.ndarray):
                    np.testing.assert_array_equal(a, b)
                else:
                    assert a == b
        prev = cur


# ---- benchmark workloads at full size ------------------------------------------

def _workload(specs, mode, ctx, chunk=None):
    xs = synth.render_many(specs)
    ns = [s.n_samples for s in specs]
    ps = [params(s.threshold, s.pre, s.post, s.ped_samples) for s in specs]
    log("oracle on %d fills" % len(specs))
    refs = oracle_many(xs, ns, ps)
    xd = synth.to_device(xs)
    fills = [make_fill(d, n, p) for d, n, p in zip(xd, ns, ps)]
    outs = [daq.alloc_out(f) for f in fills]
    log("GPU %s on %d fills" % (mode, len(specs)))
    run(ctx, mode, fills, outs)
    for i, (o, r) in enumerate(zip(outs, refs)):
        assert_same(o, r, ctx="fill %d (seed %d)" % (i, specs[i].seed))
    return refs


def test_workload_plain_single_fill(ctx):
    for mode in MODES:
        _workload(synth.config_c0(), mode, ctx)


def test_workload_16_fills_batched(ctx):
    """The benchmark's launch: the 16 fills autotuned, then replayed from graphs."""
    specs = synth.config_c1()
    xs = synth.render_many(specs)
    ns = [s.n_samples for s in specs]
    ps = [params(s.threshold, s.pre, s.post, s.ped_samples) for s in specs]
    refs = oracle_many(xs, ns, ps)
    fills = [make_fill(d, n, p) for d, n, p in zip(synth.to_device(xs), ns, ps)]
    outs = [daq.alloc_out(f) for f in fills]
    best = ctx.daq_autotune(fills, outs)
    log("autotuned: threads %d wgs %d variant %d parts %d" % (best.threads, best.wgs_per_cu, best.variant,
                                                             best.parts))
    ctx.set_graphs(True)
    for rep in range(3):
        for o in outs:
            poison_out(o)
        run(ctx, "batch", fills, outs)
        for i, (o, r) in enumerate(zip(outs, refs)):
            assert_same(o, r, ctx="rep %d fill %d (seed %d)" % (rep, i, specs[i].seed))
    assert sum(r.n_islands for r in refs) > 10_000
    ctx.set_schedule(*DEFAULT)


@pytest.mark.parametrize("sched", [(256, 4, 6, 0), (256, 8, 6, 0), (512, 2, 6, 0)],
                         ids=lambda s: "t%d_w%d_v%d_p%d" % s)
def test_workload_16_fills_pipe(ctx, sched):
    """The 16-fill launch through the persistent scan-and-copy kernel, graphs replayed."""
    specs = synth.config_c1()
    xs = synth.render_many(specs)
    ns = [s.n_samples for s in specs]
    ps = [params(s.threshold, s.pre, s.post, s.ped_samples) for s in specs]
    refs = oracle_many(xs, ns, ps)
    fills = [make_fill(d, n, p) for d, n, p in zip(synth.to_device(xs), ns, ps)]
    outs = [daq.alloc_out(f) for f in fills]
    ctx.set_schedule(*sched)
    ctx.set_graphs(True)
    for rep in range(3):
        for o in outs:
            poison_out(o)
        log("pipe 16 fills sched=%s rep=%d" % (sched, rep))
        run(ctx, "batch", fills, outs)
        for i, (o, r) in enumerate(zip(outs, refs)):
            assert_same(o, r, ctx="rep %d fill %d sched %s" % (rep, i, sched))
    ctx.set_schedule(*DEFAULT)


def test_workload_16_fills_per_fill(ctx):
    _workload(synth.config_c1(), "chop", ctx)


def test_max_channels(ctx):
    """65535 channels (the largest count whose int16 sums stay exact in int32),
    ragged length, values at both int16 extremes in places."""
    rng = np.random.default_rng(65535)
    C, N = daq.DAQ_MAX_CHANNELS, 1001
    x = rng.integers(-5, 6, size=(C, N)).astype(np.int16)
    x[:, 500:540] = -32768
    x[:, 700:710] = 32767
    x[rng.integers(0, C, 2000), rng.integers(0, N, 2000)] -= 3000
    x = pad_stride(x)
    S = x[:, :N].astype(np.int64).sum(0)
    for thr in (int(np.quantile(S, 0.05)), -(2 ** 31) + 1, 2 ** 31 - 1):
        p = params(thr, 3, 5, 20)
        ref = oracle_result(x, N, p)
        for mode in MODES:
            log("max channels thr=%d mode=%s" % (thr, mode))
            f = make_fill(dev(x), N, p)
            o = daq.alloc_out(f)
            run(ctx, mode, [f], [o])
            assert_same(o, ref, ctx="C=65535 thr %d %s" % (thr, mode))


def test_max_samples(ctx):
    """One channel of 2^31 - 1 samples (the largest fill), with pulses at known
    places near both ends and the middle; islands and packed samples are
    checked against their closed form (windows [t - pre, t + post], clipped,
    merged)."""
    N = daq.DAQ_MAX_SAMPLES
    stride = N + 1
    x = torch.full((1, stride), 1000, dtype=torch.int16, device="cuda")
    pulses = [0, 5, 1000, 1 << 30, N - 99, N - 1]
    for t in pulses:
        x[0, t] = 400
    # pedestal of the first 1000 samples: (998 * 1000 + 2 * 400) / 1000 = 998.8 -> 999
    p = params(-100, 8, 24, 1000)
    expect = [(0, 30), (992, 1025), ((1 << 30) - 8, (1 << 30) + 25), (N - 107, N - 74), (N - 9, N)]
    offs = np.cumsum([0] + [b - a for a, b in expect])
    isl_ref = np.array([(a, b, o) for (a, b), o in zip(expect, offs[:-1])], np.int64)
    out_ref = np.concatenate([np.where(np.isin(np.arange(a, b), pulses), 400, 1000) for a, b in expect])
    for mode in MODES:
        log("max samples N=%d mode=%s" % (N, mode))
        f = daq.Fill(x, N, threshold=-100, pre=8, post=24, ped_samples=1000)
        o = daq.alloc_out(f)
        run(ctx, mode, [f], [o])
        isl, n, total, status, ped, out = o.host()
        assert (n, total, status) == (len(expect), int(offs[-1]), 0), mode
        np.testing.assert_array_equal(ped, [999])
        np.testing.assert_array_equal(isl, isl_ref)
        np.testing.assert_array_equal(out[0], out_ref)
        del o
        torch.cuda.empty_cache()


def test_workload_uneven_24_streams(ctx):
    _workload(synth.config_c2(), "batch", ctx)


@pytest.mark.parametrize("sched", [DEFAULT, (256, 4, 6, 0)], ids=lambda s: "t%d_w%d_v%d_p%d" % s)
def test_workload_detector_stress(ctx, sched):
    # four whole-detector fills: 96 calorimeter units of 54 x 560,000
    ctx.set_schedule(*sched)
    _workload(synth.config_c4(), "batch", ctx)
    ctx.set_schedule(*DEFAULT)


def test_autotune_candidates_agree(ctx, tmp_path):
    if os.environ.get("DAQ_SCHEDULE"):
        pytest.skip("DAQ_SCHEDULE fixes the schedule: the tuner launches nothing")
    specs = synth.config_c1(4)
    xs = synth.render_many(specs)
    ps = [params(s.threshold, s.pre, s.post) for s in specs]
    refs = oracle_many(xs, [s.n_samples for s in specs], ps)
    xd = synth.to_device(xs)
    fills = [make_fill(d, s.n_samples, p) for d, s, p in zip(xd, specs, ps)]
    outs = [daq.alloc_out(f) for f in fills]
    log("autotune on 4 fills")
    best = ctx.daq_autotune(fills, outs, cache_path=str(tmp_path / "tune.txt"))
    torch.cuda.synchronize()
    assert best.threads in (256, 512)
    for o, r in zip(outs, refs):
        assert_same(o, r, ctx="after autotune")
    # the cached choice is reused
    best2 = ctx.daq_autotune(fills, outs, cache_path=str(tmp_path / "tune.txt"))
    assert (best2.threads, best2.wgs_per_cu, best2.variant) == (best.threads, best.wgs_per_cu, best.variant)
    ctx.set_schedule(*DEFAULT)


def test_batches_alternating_over_two_streams():
    """The benchmark's job form: consecutive batches alternate over two HIP
    streams, each stream with its own context, its own copy of the fills and
    its own outputs, so that batches overlap on the device. Every launch's
    results equal the oracle's (outputs poisoned before each launch is
    issued; the results are checked after the last one)."""
    specs = synth.config_c1(4)
    xs = synth.render_many(specs)
    ps = [params(s.threshold, s.pre, s.post) for s in specs]
    refs = oracle_many(xs, [s.n_samples for s in specs], ps)
    xd = synth.to_device(xs)
    copies = [xd, [d.clone() for d in xd]]
    ctxs = [daq.Context(0), daq.Context(0)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    try:
        for c in ctxs:
            c.set_schedule(*DEFAULT)
            c.set_graphs(False)
        fills = [[make_fill(d, s.n_samples, p) for d, s, p in zip(cp, specs, ps)] for cp in copies]
        outs = [[daq.alloc_out(f) for f in fs] for fs in fills]
        for rnd in range(3):
            log("two streams, round %d" % rnd)
            torch.cuda.synchronize()
            for k in range(2):
                for o in outs[k]:
                    poison_out(o)
            torch.cuda.synchronize()
            for i in range(6):  # launches alternate; the last two are the ones checked
                k = i % 2
                ctxs[k].daq_process_batch(fills[k], outs[k], streams[k])
            torch.cuda.synchronize()
            for k in range(2):
                for j, (o, r) in enumerate(zip(outs[k], refs)):
                    assert_same(o, r, ctx="stream %d fill %d round %d" % (k, j, rnd))
    finally:
        for c in ctxs:
            c.close()
