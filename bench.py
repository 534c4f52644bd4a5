#!/usr/bin/env python3
"""Throughput of T-method island chopping on one MI355X.

Workload: 16 synthetic calorimeter fills of 54 channels x 560,000 int16
samples (12-bit values; 700 us at 800 MSPS, Section 3 of the paper) at 3x the
nominal initial pulse rate, threshold -200 ADC on the pedestal-subtracted
calorimeter sum, pre 8 / post 24 samples. A step chops all 16 fills: island
tables, counts, pedestals and the packed raw samples of every channel, in one
persistent batched launch replayed from a captured HIP graph (schedule from
the library's autotuner). Inputs are resident in HBM before timing starts.

Printed (one JSON line): raw ADC GB/s (value) and its fraction of the HBM
peak, p50/p99 fill latency for the batched and the plain per-fill forms, the
chop launch's roofline figures timed live with HIP events over the timed
region; lines for the Q-method, the 12-bit ingest and the compression of the
chopped fills on the same data; and the CPU oracle's throughput on a bounded
sample, after the oracle has checked the first fill of every line.
"""
import argparse
import collections
import concurrent.futures as cf
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
UNEVEN = "24 uneven calorimeter streams: N ~ U{100k..560k}, rate 0.5-4x, thr -400..-150, pre 4-16, post 16-48"
STRESS = "whole detector: 4 fills x 24 calorimeters x 54 ch x 560,000, 10x rate, thr -100, pre 8, post 48"
SERVED = ("16 serving-stream fills in one launch: 54 ch x 560,000, the nominal rate, thr -200, pre 8, post 24 "
          "(the served fills' shape)")
# Fill-0 results of each line, checked against the CPU oracle in the oracle
# leg at the end: (kind, dict that receives "parity_fill0", payload).
PENDING = []
METRIC = "raw ADC GB/s island-chopped & % HBM peak; p99 fill latency, batched vs plain"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "chop_16fills_traffic.json")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def pct(vals, q):
    import numpy as np
    return float(np.percentile(np.asarray(vals, dtype=np.float64), q)) if vals else None


def kernel_sha():
    """Hash of every source the chop kernels are built from (the traffic
    file's counts apply only to the version they were taken for)."""
    from paper_1611_04959_amd.traffic import kernel_sha as sha
    return sha()


def distinct_copies(xd, k):
    """The device fills and k - 1 copies of each in memory of their own: the
    same samples (so the same islands and the same work) at other addresses,
    so that no copy is read while another one may still be cached."""
    out = list(xd)
    for _ in range(1, k):
        for x in xd:
            out.append(x.clone())
    return out


def ceiling(daq):
    """Plain HBM rates on this GPU: a streaming read of 2 GiB (daq_read_stream,
    the best of two layouts and four grid sizes; the ceiling of the summing scan) and a
    1 GiB device copy (read + write bytes), by HIP events."""
    import torch
    n = 1 << 30
    out = {}
    buf = torch.ones(n, dtype=torch.int16, device="cuda")  # 2 GiB
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    best = 0.0
    for layout in (0, 1):
        for per_cu in (4, 8, 16, 32):
            blocks = per_cu * cus
            sink = torch.empty(blocks * 4, dtype=torch.int32, device="cuda")
            for _ in range(3):
                daq.read_stream(buf, sink, blocks, layout)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(10):
                daq.read_stream(buf, sink, blocks, layout)
            b.record()
            torch.cuda.synchronize()
            rate = 2 * n * 10 / (a.elapsed_time(b) * 1e-3) / 1e9
            if rate > best:
                best, out["read_blocks_per_cu"], out["read_layout"] = rate, per_cu, layout
    out["read_gbs"] = round(best, 1)
    del buf
    # the scan's own read pattern (tiles of 4,096 samples x 54 rows, 6 rows in
    # flight) over 16 fills of 54 x 560,000, with nothing else done
    nf, C, N = 16, 54, 560_000
    raw = torch.ones(nf * C * N, dtype=torch.int16, device="cuda")
    best_t = None
    for per_cu in (4, 8, 16):
        blocks = per_cu * cus
        sink = torch.empty(blocks * 8, dtype=torch.int32, device="cuda")
        for _ in range(3):
            daq.read_tiles(raw, nf, C, N, sink, blocks)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(10):
            daq.read_tiles(raw, nf, C, N, sink, blocks)
        b.record()
        torch.cuda.synchronize()
        us = a.elapsed_time(b) * 1e3 / 10
        if best_t is None or us < best_t:
            best_t, out["tiles_blocks_per_cu"] = us, per_cu
    out["scan_pattern_us_16fills"] = round(best_t, 1)
    out["scan_pattern_gbs"] = round(2 * nf * C * N / (best_t * 1e-6) / 1e9, 1)
    # a single pass that writes the islands from the scan, modelled: the same
    # read, then a fixed 1-in-7 group pattern read again (mode 1) and also
    # written packed (mode 2), at the best grid of the plain read
    tiles = (N + 4047) // 4048
    outw = torch.empty(nf * tiles * C * 512 * 8, dtype=torch.int16, device="cuda")
    blocks = out["tiles_blocks_per_cu"] * cus
    sink = torch.empty(blocks * 8, dtype=torch.int32, device="cuda")
    for mode, key in ((1, "scan_reread_us_16fills"), (2, "scan_reread_write_us_16fills")):
        for _ in range(3):
            daq.read_tiles(raw, nf, C, N, sink, blocks, mode, outw)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(10):
            daq.read_tiles(raw, nf, C, N, sink, blocks, mode, outw)
        b.record()
        torch.cuda.synchronize()
        out[key] = round(a.elapsed_time(b) * 1e3 / 10, 1)
    pat = 0
    for lt in range(tiles):
        g0 = (lt * 4048 - 32) // 8
        pat += sum(1 for g in range(max(g0, 0), min(g0 + 512, N // 8)) if g % 70 < 11)
    out["reread_mb_16fills"] = round(nf * C * pat * 16 / 1e6, 1)
    del raw, outw
    src = torch.ones(n // 2, dtype=torch.int16, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(10):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    out["copy_gbs"] = round(2 * n * 10 / (a.elapsed_time(b) * 1e-3) / 1e9, 1)
    del src, dst
    torch.cuda.empty_cache()
    out["what"] = ("read_gbs: one streaming read of 2 GiB with 16-byte non-temporal loads (daq_read_stream); "
                   "scan_pattern_gbs: the 16 bench-shaped fills read in the chop scan's tiles and nothing else "
                   "(daq_read_tiles), raw bytes over time; scan_reread(_write)_us: the same read, then 1 in 7 "
                   "of each tile's groups read again (and written packed): a model of a single pass; "
                   "copy_gbs: torch device copy of 1 GiB, read + write bytes")
    return out


# first fills of each timed configuration (host copies, their specs), for the
# oracle's single-core rate per configuration
ORACLE_SAMPLES = {}


def batch_bench(daq, synth, specs, what, steps=20, warmup=3, name=None):
    """One batched launch over `specs` (autotuned on that batch): raw GB/s,
    the chop pass's HIP-event time, and parity of the first fill."""
    import numpy as np
    import torch
    log("batch %s: rendering %d fills" % (what.split(":")[0], len(specs)))
    xs = synth.render_many(specs)
    ORACLE_SAMPLES[name or what] = (xs[:2], specs[:2])
    xd = synth.to_device(xs)
    fills = [daq.Fill(d, sp.n_samples, threshold=sp.threshold, pre=sp.pre, post=sp.post,
                      ped_samples=sp.ped_samples) for d, sp in zip(xd, specs)]
    outs = [daq.alloc_out(f) for f in fills]
    raw = sum(sp.raw_bytes for sp in specs)
    ctx = daq.Context(0)
    best = ctx.daq_autotune(fills, outs)
    batch = daq.Batch(fills, outs)
    for _ in range(warmup):
        ctx.daq_process_batch(batch)
    torch.cuda.synchronize()
    # timed as the main batch: events only at both ends of the region, then
    # each launch between its own events for the latency percentiles
    stream = torch.cuda.current_stream()
    ev_a, ev_b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev_a.record(stream)
    for _ in range(steps):
        ctx.daq_process_batch(batch)
    ev_b.record(stream)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    launch_ms = ev_a.elapsed_time(ev_b) / steps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record(stream)
        ctx.daq_process_batch(batch)
        b.record(stream)
    torch.cuda.synchronize()
    step_ms = [a.elapsed_time(b) for a, b in ev]
    cnt = torch.stack([o.counts for o in outs]).cpu().numpy()
    tot = int(cnt[:, 1].sum())
    alg = sum(2 * sp.n_channels * sp.n_samples for sp in specs) \
        + sum(2 * sp.n_channels * int(t) + 24 * int(n) + 24 + 4 * sp.n_channels
              for sp, n, t in zip(specs, cnt[:, 0], cnt[:, 1]))
    graphs = ctx.get_graphs()
    ctx.close()
    res = {"workload": what, "fills": len(specs), "raw_gb": round(raw / 1e9, 3),
           "seeds": [sp.seed for sp in specs], "islands": [int(v) for v in cnt[:, 0]],
           "ms_per_step": round(ms, 4), "gbs": round(raw / (ms * 1e-3) / 1e9, 1),
           "pct_hbm_peak": round(100 * raw / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 2),
           "kernel_ms_mean": round(launch_ms, 4),
           "algorithmic_bytes_per_launch": int(alg),
           "algorithmic_gbs": round(alg / (launch_ms * 1e-3) / 1e9, 1),
           "p50_fill_ms": round(pct(step_ms, 50), 4), "p99_fill_ms": round(pct(step_ms, 99), 4),
           "occupancy": round(tot / sum(sp.n_samples for sp in specs), 4),
           "schedule": {"threads": best.threads, "wgs_per_cu": best.wgs_per_cu, "variant": best.variant,
                        "parts": best.parts, "graphs": graphs},
           "steps": steps, "parity_fill0": None}
    PENDING.append(("chop", res, (xs[0], specs[0], outs[0].host())))
    del xd, fills, outs
    torch.cuda.empty_cache()
    return res


def plain_c0_bench(daq, synth, ctx, rounds=10):
    """The plain form at the single-fill shape: eight 54 x 560,000 fills at the
    nominal rate (distinct seeds, 484 MB together, more than the 256 MB
    last-level cache), one daq_chop_fill call each, in turn; per-call latency
    by HIP events around each call."""
    import numpy as np
    import torch
    specs = [synth.config_c0(i)[0] for i in range(8)]
    xs = synth.render_many(specs)
    ORACLE_SAMPLES["c0"] = (xs[:2], specs[:2])
    xd = synth.to_device(xs)
    fills = [daq.Fill(d, sp.n_samples, threshold=sp.threshold, pre=sp.pre, post=sp.post,
                      ped_samples=sp.ped_samples) for d, sp in zip(xd, specs)]
    outs = [daq.alloc_out(f) for f in fills]
    st = torch.cuda.current_stream()
    for f, o in zip(fills, outs):
        ctx.daq_chop_fill(f, o, st)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(rounds * len(fills))]
    t0 = time.perf_counter()
    for r in range(rounds):
        for i, (f, o) in enumerate(zip(fills, outs)):
            a, b = ev[r * len(fills) + i]
            a.record(st)
            ctx.daq_chop_fill(f, o, st)
            b.record(st)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / (rounds * len(fills))
    lat = [a.elapsed_time(b) for a, b in ev]
    cnt = torch.stack([o.counts for o in outs]).cpu().numpy()
    alg = sum(2 * sp.n_channels * sp.n_samples + 2 * sp.n_channels * int(t) + 24 * int(n) + 24 + 4 * sp.n_channels
              for sp, n, t in zip(specs, cnt[:, 0], cnt[:, 1]))
    res = {"workload": "plain form, one call per fill: 8 fills of 54 ch x 560,000 at the nominal rate "
                       "(thr -200, pre 8, post 24), distinct seeds, taken in turn",
           "seeds": [sp.seed for sp in specs], "islands": [int(v) for v in cnt[:, 0]],
           "occupancy": round(float(cnt[:, 1].sum()) / sum(sp.n_samples for sp in specs), 4),
           "ms_per_fill": round(ms, 4), "gbs": round(specs[0].raw_bytes / (ms * 1e-3) / 1e9, 1),
           "algorithmic_gbs": round(alg / len(specs) / (ms * 1e-3) / 1e9, 1),
           "p50_fill_ms": round(pct(lat, 50), 4), "p99_fill_ms": round(pct(lat, 99), 4),
           "parity_fill0": None}
    PENDING.append(("chop", res, (xs[0], specs[0], outs[0].host())))
    del xd, fills, outs
    torch.cuda.empty_cache()
    return res


def arrivals(rate, seconds, rng, burst_x=5.0, burst_s=0.080, duty=0.10):
    """Arrival times (s) of a Poisson process of long-run mean `rate` per second
    whose rate is burst_x times higher inside bursts of burst_s seconds that
    take a fraction `duty` of the time (the base rate is lowered to keep the
    mean)."""
    base = rate / (1.0 - duty + burst_x * duty)
    period = burst_s / duty
    t, out = 0.0, []
    while t < seconds:
        in_burst = (t % period) < burst_s
        lam = base * (burst_x if in_burst else 1.0)
        # thinning against the burst rate keeps the process exact at the edges
        t += rng.exponential(1.0 / (base * burst_x))
        if rng.random() < lam / (base * burst_x) and t < seconds:
            out.append(t)
    return out


def q_bench(daq, ctx, xs, fills, specs, steps, warmup):
    """The Q-method on the same 16 fills: decimated sums and fill-by-fill accumulators
    (one daq_qmethod_batch call per step, every fill adding into its own accumulator)."""
    import numpy as np
    import torch
    qs = [daq.alloc_q_out(f) for f in fills]
    for _ in range(warmup):
        ctx.daq_qmethod_batch(fills, qs)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        ctx.daq_qmethod_batch(fills, qs)
    e1.record()
    torch.cuda.synchronize()
    kt = ctx.kernel_times_ms()
    ctx.set_timing(False)
    ms = e0.elapsed_time(e1) / steps
    kms = float(np.mean(kt)) if kt else ms
    raw = sum(s.raw_bytes for s in specs)
    acc_bytes = sum(2 * 4 * s.n_samples * x.shape[0] for s, x in zip(specs, xs))   # read + write
    q_bytes = sum(8 * ((s.n_samples + 31) // 32) for s in specs)
    alg = raw + acc_bytes + q_bytes
    res = {}
    PENDING.append(("qmethod", res, (xs[0], specs[0], warmup + steps, qs[0].qsum.cpu().numpy(),
                                     qs[0].acc[:, :specs[0].n_samples].cpu().numpy())))
    res.update({"workload": "Q-method on the same %d fills: decimated sum (bins of 32) and an int32 "
                            "fill-by-fill accumulator per fill, one call per step" % len(specs),
                "steps": steps, "ms_per_step": round(ms, 4), "raw_gbs": round(raw / ms / 1e6, 1),
                "kernel_ms_mean": round(kms, 4),
                "roofline": {"bound": "hbm", "achieved": round(alg / kms / 1e6, 1), "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": round(alg / kms / 1e6 / HBM_PEAK_GBS, 4),
                             "kernel": "k_q_pass", "algorithmic_bytes_per_launch": alg},
                "parity_fill0": None})
    return res


def oracle_check(oracle, kind, payload) -> bool:
    """Fill 0 of one line against the oracle: the chop (records, pedestals, packed rows),
    the Q-method after k calls (sums; accumulator modulo 2^32) or the compressed stream."""
    import numpy as np

    def chop(x, sp):
        return oracle.chop(x, n_samples=sp.n_samples, ped_samples=sp.ped_samples, threshold=sp.threshold,
                           pre=sp.pre, post=sp.post)

    if kind == "chop":
        x, sp, (isl, n, total, st, ped, out) = payload
        ref = chop(x, sp)
        return bool(n == ref.n_islands and total == ref.total_len and st == 0 and
                    np.array_equal(isl, ref.islands) and np.array_equal(ped, ref.ped) and
                    np.array_equal(out, ref.out))
    if kind == "qmethod":
        x, sp, k, qsum, acc = payload
        N = sp.n_samples
        ped, Q = oracle.qmethod(x, N, ped_samples=sp.ped_samples)
        want = (k * (x[:, :N].astype(np.int64) - ped[:, None].astype(np.int64))) % 2**32
        return bool(np.array_equal(qsum, Q) and np.array_equal(want, acc.astype(np.int64) % 2**32))
    if kind == "fig2":
        x, x0, sp, thrs, found, truth = payload
        want = [[chop(h, dataclasses.replace(sp, threshold=t)).n_islands for t in thrs] for h in (x, x0)]
        return want == [list(found), list(truth)]
    if kind == "tq":
        x, sp, k, (isl, n, total, st, ped, out), qsum, acc = payload
        ref = chop(x, sp)
        N = sp.n_samples
        qped, Q = oracle.qmethod(x, N, ped_samples=sp.ped_samples)
        want = (k * (x[:, :N].astype(np.int64) - qped[:, None].astype(np.int64))) % 2**32
        return bool(n == ref.n_islands and total == ref.total_len and st == 0 and
                    np.array_equal(isl, ref.islands) and np.array_equal(ped, ref.ped) and
                    np.array_equal(out, ref.out) and np.array_equal(qsum, Q) and
                    np.array_equal(want, acc.astype(np.int64) % 2**32))
    if kind == "compress":
        x, sp, hdr, words = payload
        ref = chop(x, sp)
        hdr_ref, words_ref = oracle.z_compress(ref.out, ref.total_len)
        return bool(np.array_equal(hdr, hdr_ref) and np.array_equal(words, words_ref))
    raise ValueError(kind)


def z_bench(daq, ctx, outs, x0, spec0, steps, warmup=3):
    """Lossless compression of the 16 chopped fills (per-block delta, zigzag and bit
    width), one daq_compress_batch call per step over the packed rows of the last launch;
    then one daq_decompress_batch call per step decoding the streams back."""
    import numpy as np
    import torch
    C = int(outs[0].out.shape[0])
    zouts = [daq.alloc_z_out(C, int(o.out.shape[1]), device="cuda") for o in outs]
    for _ in range(warmup):
        ctx.daq_compress_batch(outs, zouts)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        ctx.daq_compress_batch(outs, zouts)
    e1.record()
    torch.cuda.synchronize()
    kt = ctx.kernel_times_ms()
    ctx.set_timing(False)
    ms = e0.elapsed_time(e1) / steps
    kms = float(np.mean(kt)) if kt else ms
    tot = [int(o.counts[1].item()) for o in outs]
    packed = sum(2 * C * t for t in tot)
    blocks = sum(C * ((t + 63) // 64) for t in tot)
    n_words = sum(int(z.n_words.item()) for z in zouts)
    alg = packed + 12 * blocks + 4 * n_words          # samples read; headers, offsets, payload written
    stream_bytes = 4 * blocks + 4 * n_words           # what leaves the frontend: headers and payload
    # decoding the same streams back into packed rows
    backs = [torch.empty_like(o.out) for o in outs]
    for _ in range(warmup):
        ctx.daq_decompress_batch(zouts, tot, backs)
    torch.cuda.synchronize()
    d0, d1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    d0.record()
    for _ in range(steps):
        ctx.daq_decompress_batch(zouts, tot, backs)
    d1.record()
    torch.cuda.synchronize()
    dms = d0.elapsed_time(d1) / steps
    round_trip = all(torch.equal(b[:, :t], o.out[:, :t]) for b, o, t in zip(backs, outs, tot))
    dec_alg = packed + 12 * blocks + 4 * n_words      # payload, headers and offsets read; samples written
    res = {}
    hdr0, _, words0 = zouts[0].host(C, tot[0])
    PENDING.append(("compress", res, (x0, spec0, hdr0, words0)))
    res.update({"workload": "lossless compression of the %d chopped fills' packed rows (blocks of 64: "
                            "first sample, bit width, zigzag deltas), one call per step" % len(outs),
                "steps": steps, "ms_per_step": round(ms, 4), "packed_gbs": round(packed / ms / 1e6, 1),
                "kernel_ms_mean": round(kms, 4), "ratio": round(packed / stream_bytes, 3),
                "bits_per_sample": round(8 * stream_bytes / (packed / 2), 3),
                "roofline": {"bound": "hbm", "achieved": round(alg / kms / 1e6, 1), "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": round(alg / kms / 1e6 / HBM_PEAK_GBS, 4),
                             "kernel": "one call: k_z_size, k_z_pack",
                             "algorithmic_bytes_per_launch": alg},
                "decompress": {"ms_per_step": round(dms, 4), "packed_gbs": round(packed / dms / 1e6, 1),
                               "algorithmic_gbs": round(dec_alg / dms / 1e6, 1),
                               "frac": round(dec_alg / dms / 1e6 / HBM_PEAK_GBS, 4), "kernel": "k_unz",
                               "round_trip_exact": bool(round_trip)},
                "parity_fill0": None})
    return res


FIG2_KS = [0.5, 1, 2, 3, 4, 6, 10, 20]


def fig2_bench(daq, synth, ctx, n_fills=16):
    """A Figure 2 analog: islands found against true islands at thresholds k sigma below
    each fill's baseline, for 16 fills at the nominal rate. Truth is the same chop of the
    noiseless rendering (the generator's noise is counter-based: the pulses stay put).
    The baselines come from the device's Q-method sums; the whole sweep (noisy and
    noiseless, every threshold) is one batched launch over shared raw rows."""
    import numpy as np
    import torch
    specs = [synth.FillSpec(seed=synth.fill_seed("fig2", 0, i)) for i in range(n_fills)]
    N = specs[0].n_samples
    sigma = 3.0 * float(np.sqrt(synth.CHANNELS))
    xs = synth.render_many(specs)
    x0s = [synth.render(sp, noise_sigma=0.0) for sp in specs]
    xd, x0d = synth.to_device(xs), synth.to_device(x0s)
    base = [daq.Fill(d, N, ped_samples=sp.ped_samples) for d, sp in zip(xd, specs)]
    qs = [daq.alloc_q_out(f, acc=False) for f in base]
    ctx.daq_qmethod_batch(base, qs)
    torch.cuda.synchronize()
    b = [int(np.median(q.qsum.cpu().numpy()[:N // daq.DAQ_Q_DECIMATION]) // daq.DAQ_Q_DECIMATION) for q in qs]
    thr = [[int(bi - k * sigma) for k in FIG2_KS] for bi in b]
    fills, outs = [], []
    for raws in (xd, x0d):
        for i, d in enumerate(raws):
            for t in thr[i]:
                fills.append(daq.Fill(d, N, threshold=t, pre=8, post=24, ped_samples=100))
                outs.append(daq.alloc_out(fills[-1]))
    ctx.daq_process_batch(fills, outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.daq_process_batch(fills, outs)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    counts = np.array([int(o.counts[0].item()) for o in outs]).reshape(2, n_fills, len(FIG2_KS))
    found, truth = counts[0].sum(0), counts[1].sum(0)
    # per true pulse (the generator's list): found when its start lies in an island of the
    # noisy fill; pulses deeper than 1.5 times the threshold's depth, and all pulses
    eff_deep, eff_all = np.zeros(len(FIG2_KS)), np.zeros(len(FIG2_KS))
    n_deep, n_all = np.zeros(len(FIG2_KS)), np.zeros(len(FIG2_KS))
    for i, sp in enumerate(specs):
        _, pulses = synth.render(sp, truth=True)
        for kk, k in enumerate(FIG2_KS):
            o = outs[i * len(FIG2_KS) + kk]
            n_isl = min(int(o.counts[0].item()), int(o.islands.shape[0]))
            isl = o.islands[:n_isl].cpu().numpy()
            j = np.searchsorted(isl[:, 0], pulses["t0"], side="right") - 1
            inside = (j >= 0) & (pulses["t0"] < isl[np.maximum(j, 0), 1]) if n_isl else np.zeros(len(pulses), bool)
            deep = pulses["amp"] >= 1.5 * k * sigma
            eff_deep[kk] += inside[deep].sum()
            n_deep[kk] += deep.sum()
            eff_all[kk] += inside.sum()
            n_all[kk] += len(pulses)
    res = {"workload": "Figure 2 analog: %d fills x 54 ch x 560,000 at the nominal rate, thresholds k sigma "
                       "below each fill's baseline (sigma = %.1f ADC, the summed noise), islands found vs "
                       "the same chop of the noiseless rendering; one launch of %d entries"
                       % (n_fills, sigma, len(fills)),
           "k_sigma": FIG2_KS, "found": found.tolist(), "truth": truth.tolist(),
           "ratio": [round(float(f) / max(float(t), 1.0), 4) for f, t in zip(found, truth)],
           "pulse_efficiency_deep": [round(float(e) / max(float(n), 1.0), 4) for e, n in zip(eff_deep, n_deep)],
           "pulse_efficiency_all": [round(float(e) / max(float(n), 1.0), 4) for e, n in zip(eff_all, n_all)],
           "ms_per_sweep": round(ms, 3), "parity_fill0": None}
    PENDING.append(("fig2", res, (xs[0], x0s[0], specs[0], thr[0], counts[0][0].tolist(), counts[1][0].tolist())))
    del xd, x0d, fills, outs, base, qs
    torch.cuda.empty_cache()
    return res


def tq_bench(daq, ctx, xs, fills, specs, steps, warmup=2):
    """Both methods on the 16 fills: one daq_process_batch_q call (the Q-method inside the chop's
    scan pass, one read of the raw samples) against daq_process_batch then daq_qmethod_batch."""
    import numpy as np
    import torch
    outs = [daq.alloc_out(f) for f in fills]
    qs = [daq.alloc_q_out(f) for f in fills]
    for q in qs:
        q.ped = None
    outs2 = [daq.alloc_out(f) for f in fills]
    qs2 = [daq.alloc_q_out(f) for f in fills]

    def fused():
        ctx.daq_process_batch_q(fills, outs, qs)

    def separate():
        ctx.daq_process_batch(fills, outs2)
        ctx.daq_qmethod_batch(fills, qs2)

    res = {}
    for name, fn in (("fused", fused), ("separate", separate)):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        res[name] = e0.elapsed_time(e1) / steps
    tot = [int(o.counts[1].item()) for o in outs]
    n_isl = [int(o.counts[0].item()) for o in outs]
    C = xs[0].shape[0]
    raw = sum(s.raw_bytes for s in specs)
    acc_bytes = sum(2 * 4 * s.n_samples * x.shape[0] for s, x in zip(specs, xs))
    alg = raw + acc_bytes + sum(8 * ((s.n_samples + 31) // 32) for s in specs) + sum(2 * C * t for t in tot) \
        + sum(24 * n for n in n_isl)
    out = {"workload": "T-method and Q-method on the same %d fills: daq_process_batch_q (one read of the raw "
                       "samples) against daq_process_batch followed by daq_qmethod_batch" % len(fills),
           "steps": steps, "fused_ms": round(res["fused"], 4), "separate_ms": round(res["separate"], 4),
           "speedup": round(res["separate"] / res["fused"], 3),
           "fused_algorithmic_gbs": round(alg / res["fused"] / 1e6, 1),
           "fused_pct_hbm_peak": round(100 * alg / res["fused"] / 1e6 / HBM_PEAK_GBS, 2),
           "algorithmic_bytes_per_call": alg, "parity_fill0": None}
    k = warmup + steps
    PENDING.append(("tq", out, (xs[0], specs[0], k, outs[0].host(), qs[0].qsum.cpu().numpy(),
                                qs[0].acc[:, :specs[0].n_samples].cpu().numpy())))
    del outs, qs, outs2, qs2
    torch.cuda.empty_cache()
    return out


def ingest12_bench(daq, ctx, xs, specs, steps):
    """12-bit ingest: the 16 fills as packed digitizer words (two samples to three bytes),
    unpacked on the device; and host-to-device copies of packed and int16 rows from
    pinned memory, which bound a host-fed DAQ."""
    import numpy as np
    import torch
    N = specs[0].n_samples
    C = xs[0].shape[0]
    nb = (3 * N + 1) // 2
    pst = (nb + 3) // 4 * 4
    packed = []
    for x in xs:
        v = x[:, :N].astype(np.uint32) & 0xFFF
        if N % 2:
            v = np.concatenate([v, np.zeros((C, 1), np.uint32)], axis=1)
        a, b = v[:, 0::2], v[:, 1::2]
        trip = np.stack([a & 0xFF, (a >> 8) | ((b & 0xF) << 4), b >> 4], axis=2).reshape(C, -1)
        p = np.zeros((C, pst), np.uint8)
        p[:, :nb] = trip[:, :nb]
        packed.append(p)
    dp = [torch.from_numpy(p).cuda() for p in packed]
    raws = [torch.empty((C, x.shape[1]), dtype=torch.int16, device="cuda") for x in xs]
    for p, r in zip(dp, raws):
        ctx.daq_unpack12(p, N, r)
    torch.cuda.synchronize()
    exact = all(np.array_equal(r[:, :N].cpu().numpy(), x[:, :N]) for r, x in zip(raws[:2], xs[:2]))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        for p, r in zip(dp, raws):
            ctx.daq_unpack12(p, N, r)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    samples = len(xs) * C * N
    alg = samples * 3.5   # 1.5 bytes read, 2 written per sample
    # host-to-device copies from pinned memory (one fill, repeated)
    hp = torch.from_numpy(packed[0]).pin_memory()
    hr = torch.from_numpy(np.ascontiguousarray(xs[0])).pin_memory()
    rates = {}
    for name, h in (("packed", hp), ("int16", hr)):
        d = torch.empty_like(h, device="cuda")
        d.copy_(h, non_blocking=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(20):
            d.copy_(h, non_blocking=True)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / 20 / 1e3
        rates[name] = {"gbs": round(h.numel() * h.element_size() / t / 1e9, 1),
                       "msamples_per_s": round(C * N / t / 1e6, 1)}
    del dp, raws
    return {"workload": "the %d fills as 12-bit words (%.1f MB packed), unpacked on the device" %
                        (len(xs), sum(p.nbytes for p in packed) / 1e6),
            "ms_per_step": round(ms, 4), "raw_gbs": round(samples * 2 / ms / 1e6, 1),
            "roofline": {"bound": "hbm", "achieved": round(alg / ms / 1e6, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(alg / ms / 1e6 / HBM_PEAK_GBS, 4),
                         "kernel": "k_unpack12 (16 calls)", "algorithmic_bytes_per_step": int(alg)},
            "h2d_pinned": rates, "exact": exact}


def serve_bench(daq, synth, ctx, seconds, budget_gb=32.0, n_streams=3, max_batch=16, saturation_only=False):
    """Serving loop on 24 calorimeter streams of plain-workload fills.

    Fills are pre-staged in HBM (one per stream, standing in for a NIC/DMA
    writing into resident slots); arrivals follow a Poisson process of
    24 x 12 fills per 1.4 s on average with 5x bursts. A fill's latency runs
    from its arrival (admission waits included) to its results being ready in
    device memory. A second run offers fills as fast as the budget admits them
    (saturation), and a third feeds fills from pinned host memory (ingest over
    PCIe, reported apart)."""
    import numpy as np
    import torch
    n_streams_in = 24
    specs = [synth.config_c3_fill(s, 0) for s in range(n_streams_in)]
    log("serving: rendering %d stream fills" % len(specs))
    xs = synth.render_many(specs)
    ORACLE_SAMPLES["c3"] = (xs[:2], specs[:2])
    # a pool of distinct fills in HBM, far larger than what is in flight, so
    # that no fill is read while its previous copy may still be cached: each
    # rendered fill and seven copies of it in memory of their own
    xd = distinct_copies(synth.to_device(xs), 8)
    sp0 = specs[0]
    fills = [daq.Fill(d, sp0.n_samples, threshold=sp0.threshold, pre=sp0.pre, post=sp0.post,
                      ped_samples=sp0.ped_samples) for d in xd]
    n_pool = len(fills)
    raw = specs[0].raw_bytes
    C = synth.CHANNELS
    arena = torch.empty(int(budget_gb * 1e9), dtype=torch.uint8, device="cuda")
    srv = daq.Server(ctx, arena, n_streams=n_streams, max_batch=max_batch)

    def run(times, host=None, dur=5.0, depth=96, packed=False):
        """Open loop: offers fills at `times` (s). Closed loop (times None):
        keeps `depth` fills submitted and unfinished for `dur` seconds."""
        pending = collections.deque()  # (arrival_ns, stream) not yet admitted
        arr_ns = {}
        kept = None
        st0 = srv.stats()
        lat, done_bytes, alg_bytes, island_samples = [], 0, 0, 0
        t0 = time.monotonic_ns()
        i, n_off = 0, 0
        end_ns = t0 + int(dur * 1e9)
        while True:
            now = time.monotonic_ns()
            if times is not None:
                while i < len(times) and t0 + int(times[i] * 1e9) <= now:
                    pending.append((t0 + int(times[i] * 1e9), i % n_pool))
                    i += 1
            else:
                while now < end_ns and len(pending) + len(arr_ns) < depth:
                    pending.append((now, n_off % n_pool))
                    n_off += 1
            while pending:
                a_ns, st = pending[0]
                if host is None:
                    t = srv.submit(fills[st], tag=st, arrival_ns=a_ns)
                elif packed:
                    t = srv.submit(fills[st], tag=st, host_packed12=host[st % len(host)], arrival_ns=a_ns)
                else:
                    t = srv.submit(fills[st], tag=st, host_raw=host[st % len(host)], arrival_ns=a_ns)
                if t is None:
                    break
                arr_ns[t] = a_ns
                pending.popleft()
            for c in srv.poll(256, 200):
                assert c.error == 0 and c.status == 0
                lat.append((c.t_ready_ns - arr_ns.pop(c.ticket)) * 1e-6)
                done_bytes += raw
                # as the batched line counts them: raw read, packed samples,
                # records, counts and pedestals written
                alg_bytes += raw + 2 * C * c.total_len + 24 * c.n_islands + 24 + 4 * C
                island_samples += c.total_len
                # the first completion whose samples are a rendered fill is kept
                # (its slot unreleased) for the oracle check after the run
                data = (c.tag % len(host)) if host is not None else (c.tag if c.tag < len(xs) else None)
                if kept is None and data is not None:
                    kept = (c, data)
                else:
                    srv.release(c.ticket)
            if times is not None and i >= len(times) and not pending and not arr_ns:
                break
            if times is None and now >= end_ns and not pending and not arr_ns:
                break
        wall = (time.monotonic_ns() - t0) * 1e-9
        st = srv.stats()
        res = {"fills": len(lat), "p50_ms": round(pct(lat, 50), 4), "p99_ms": round(pct(lat, 99), 4),
               "max_ms": round(max(lat), 4), "gbs": round(done_bytes / wall / 1e9, 1),
               "pct_hbm_peak": round(100 * done_bytes / wall / 1e9 / HBM_PEAK_GBS, 2),
               "algorithmic_gbs": round(alg_bytes / wall / 1e9, 1),
               "pct_hbm_peak_algorithmic": round(100 * alg_bytes / wall / 1e9 / HBM_PEAK_GBS, 2),
               "occupancy": round(island_samples / max(1, len(lat) * specs[0].n_samples), 4),
               "wall_s": round(wall, 2), "batches": int(st.batches - st0.batches),
               # high-water mark of the arena since the server started (all runs so far)
               "arena_high_water_gb": round(st.arena_peak / 1e9, 2),
               "late_fills": int(st.late - st0.late), "deadtime_ms": round((st.deadtime_ns - st0.deadtime_ns) / 1e6, 3),
               "refused_submits": int(st.rejected - st0.rejected), "timed_out": int(st.timed_out - st0.timed_out),
               "parity_fill0": None}
        if kept is not None:
            c, data = kept
            isl, ped, out = srv.results(c, synth.CHANNELS)
            PENDING.append(("chop", res, (xs[data], specs[data],
                                          (isl, c.n_islands, c.total_len, c.status, ped, out))))
            srv.release(c.ticket)
        return res

    rate = 24 * 12 / 1.4
    rng = np.random.default_rng(3)
    if saturation_only:  # the saturation line alone, for `seconds` (profiling)
        sat = run(None, dur=seconds, depth=96)
        srv.close()
        del arena
        torch.cuda.empty_cache()
        return {"workload": "serving loop at saturation (96 fills in flight), %.1f s" % seconds, "saturation": sat}
    # long enough for p50 / p99 over at least 10,000 fills
    nominal_s = max(seconds, 10_000 / rate * 1.03)
    times = arrivals(rate, nominal_s, rng)
    log("serving: %d arrivals over %.0f s (mean %.1f fills/s, 5x bursts)" % (len(times), nominal_s, rate))
    nominal = run(times)
    # the other reading of the rate: 12 fills per second on every stream
    rate12 = 24 * 12.0
    s12 = max(seconds, 10_000 / rate12 * 1.03)
    log("serving: 12 Hz per stream, %.0f s" % s12)
    nominal_12hz = run(arrivals(rate12, s12, rng))
    nominal_12hz["offered_fills_per_s"] = rate12  # in place: the parity check fills this dict later
    log("serving: saturation (96 fills kept in flight)")
    sat = run(None, depth=96)
    # open loop at multiples of the nominal rate, until the queue grows
    sweep = []
    for k in (50, 100, 200, 300, 400):
        log("serving: open loop at %dx the nominal rate" % k)
        r = run(arrivals(rate * k, 2.0, rng))
        r["offered_fills_per_s"] = round(rate * k, 1)
        r["offered_gbs"] = round(rate * k * specs[0].raw_bytes / 1e9, 1)
        sweep.append(r)
    ingest = None
    try:
        host = [torch.from_numpy(x).pin_memory() for x in xs[:8]]
        log("serving: host-fed ingest at the nominal rate, then saturated")
        ingest = {"nominal": run(arrivals(rate, 5.0, rng), host=host),
                  "saturation": run(None, host=host, depth=32)}
        N = specs[0].n_samples
        if all(0 <= int(x.min()) and int(x.max()) <= 4095 for x in xs[:8]):
            pst = daq.packed12_stride(N)
            hp = []
            for x in xs[:8]:
                v = x[:, :N].astype(np.uint32) & 0xFFF
                if N % 2:
                    v = np.concatenate([v, np.zeros((v.shape[0], 1), np.uint32)], axis=1)
                a, b = v[:, 0::2], v[:, 1::2]
                trip = np.stack([a & 0xFF, (a >> 8) | ((b & 0xF) << 4), b >> 4], axis=2).reshape(v.shape[0], -1)
                p = np.zeros((x.shape[0], pst), np.uint8)
                p[:, :(3 * N + 1) // 2] = trip[:, :(3 * N + 1) // 2]
                hp.append(torch.from_numpy(p).pin_memory())
            log("serving: host-fed 12-bit words at the nominal rate, then saturated")
            ingest["nominal_packed12"] = run(arrivals(rate, 5.0, rng), host=hp, packed=True)
            ingest["saturation_packed12"] = run(None, host=hp, depth=32, packed=True)
    except RuntimeError as e:  # pinned memory unavailable
        log("ingest skipped: %s" % e)
    srv.close()
    del arena
    torch.cuda.empty_cache()
    return {"workload": "24 streams of 54 ch x 560,000 int16 fills (plain-workload shape), fills pre-staged "
                        "in HBM; Poisson arrivals, 24 x 12 fills per 1.4 s on average with 5x bursts "
                        "(80 ms, 10 % duty)", "offered_fills_per_s": round(rate, 1),
            "budget_gb": budget_gb, "n_streams": n_streams, "max_batch": max_batch,
            "seeds": [sp.seed for sp in specs],
            "nominal": nominal, "nominal_12hz": nominal_12hz,
            "saturation": sat, "open_loop": sweep, "ingest_pcie": ingest}


def island_line_bytes(records, row_bases, line=128):
    """Bytes of the `line`-byte cache lines that hold island samples: records
    is one (n, 2) array of [start, stop) per fill, row_bases the byte address
    of each of that fill's int16 channel rows. Islands never overlap but two
    may end and begin in one line, which is counted once. Any kernel that
    reads the island samples from the raw rows fetches at least this much."""
    import numpy as np
    total = 0
    for rec, bases in zip(records, row_bases):
        rec = np.asarray(rec, np.int64).reshape(-1, 2)
        if rec.shape[0] == 0:
            continue
        for b in np.asarray(bases, np.int64):
            first = (b + 2 * rec[:, 0]) // line
            last = (b + 2 * rec[:, 1] - 1) // line
            shared = int(np.count_nonzero(first[1:] == last[:-1]))
            total += (int((last - first + 1).sum()) - shared) * line
    return total


def cpu_model():
    """The host CPU's model name (empty where /proc/cpuinfo does not say)."""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def device_info():
    """Name, architecture, compute units and memory of GPU 0."""
    import torch
    props = torch.cuda.get_device_properties(0)
    return {"name": props.name, "arch": getattr(props, "gcnArchName", ""),
            "compute_units": props.multi_processor_count, "memory_gib": round(props.total_memory / 2 ** 30, 1),
            "torch": torch.__version__, "hip": getattr(torch.version, "hip", None)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--fills", type=int, default=16)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="wall-clock budget of the CPU oracle sample (0 = skip)")
    ap.add_argument("--no-plain", action="store_true", help="skip the per-fill comparison")
    ap.add_argument("--no-tune", action="store_true", help="keep the default schedule")
    ap.add_argument("--serve-seconds", type=float, default=20.0,
                    help="serving loop at the nominal arrival rate (0 = skip)")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven-batch line")
    ap.add_argument("--no-served-shape", action="store_true",
                    help="skip the batched line over 16 fills of the serving streams' shape")
    ap.add_argument("--no-pipelined", action="store_true", help="skip the two-stream batched line")
    ap.add_argument("--no-qmethod", action="store_true", help="skip the Q-method line")
    ap.add_argument("--no-ingest", action="store_true", help="skip the 12-bit ingest line")
    ap.add_argument("--no-compress", action="store_true", help="skip the compression line")
    ap.add_argument("--no-fig2", action="store_true", help="skip the Figure 2 analog")
    ap.add_argument("--no-tq", action="store_true", help="skip the fused T-method + Q-method line")
    ap.add_argument("--no-stress", action="store_true",
                    help="skip the whole-detector stress batch (96 calorimeter fills, 5.8 GB)")
    ap.add_argument("--only-serving-saturation", action="store_true",
                    help="run only the serving loop at saturation for --serve-seconds (for profiling)")
    ap.add_argument("--only-batch", choices=["uneven", "stress"], default=None,
                    help="time only that batch shape and print its line (for profiling)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library runs on one device and has no multi-GPU path "
              "(fills are independent units, so a detector shards by calorimeter). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1611_04959_amd as daq
    import synth

    if args.only_batch:
        what = {"uneven": (synth.config_c2(), UNEVEN), "stress": (synth.config_c4(), STRESS)}[args.only_batch]
        print(json.dumps(batch_bench(daq, synth, what[0], what[1], steps=args.steps, warmup=args.warmup)), flush=True)
        return
    if args.only_serving_saturation:
        ctx = daq.Context(0)
        res = serve_bench(daq, synth, ctx, args.serve_seconds, saturation_only=True)
        ctx.close()
        print(json.dumps(res), flush=True)
        return

    specs = synth.config_c1(args.fills)
    C, N = synth.CHANNELS, specs[0].n_samples
    raw_bytes = sum(s.raw_bytes for s in specs)
    log("rendering %d fills (%.1f MB raw)" % (len(specs), raw_bytes / 1e6))
    xs = synth.render_many(specs)
    xd = synth.to_device(xs)
    fills = [daq.Fill(d, s.n_samples, threshold=s.threshold, pre=s.pre, post=s.post,
                      ped_samples=s.ped_samples) for d, s in zip(xd, specs)]
    outs = [daq.alloc_out(f) for f in fills]
    stream = torch.cuda.current_stream()
    ctx = daq.Context(0)

    # ---- schedule ---------------------------------------------------------
    if not args.no_tune:
        log("autotuning the chop schedule")
        best = ctx.daq_autotune(fills, outs)
        sched = (best.threads, best.wgs_per_cu, best.variant, best.parts)
    else:
        s = ctx.get_schedule()
        sched = (s.threads, s.wgs_per_cu, s.variant, s.parts)
    graphs = ctx.get_graphs()  # the tuner's choice of graph replay or plain launches
    log("schedule threads=%d wgs_per_cu=%d variant=%d parts=%d" % sched + (", graphs" if graphs else ", plain launches"))

    # ---- batched: warm-up then the timed region --------------------------------
    batch = daq.Batch(fills, outs)  # argument arrays built once
    for _ in range(args.warmup):
        ctx.daq_process_batch(batch, stream=stream)
    torch.cuda.synchronize()
    # the timed region: K launches between two HIP events on the launch
    # stream (their interval over K is the average launch duration, each
    # launch one graph holding all kernels of the pass); no event inside the
    # region, since every event record adds a few microseconds per step
    ev_a, ev_b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    log("timing %d batched steps" % args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev_a.record(stream)
    for k in range(args.steps):
        ctx.daq_process_batch(batch, stream=stream)
    ev_b.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    launch_ms = ev_a.elapsed_time(ev_b) / args.steps
    value = raw_bytes / (ms_per_step * 1e-3) / 1e9
    # latency of each launch (every fill of a launch completes with it): the
    # same launches again, each between its own pair of events
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    for k in range(args.steps):
        ev[k][0].record(stream)
        ctx.daq_process_batch(batch, stream=stream)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    step_ms = [a.elapsed_time(b) for a, b in ev]
    # the library's own per-launch timing (event pairs around each launch,
    # which cost a few microseconds each), in a separate short run
    ctx.set_timing(True)
    for _ in range(max(5, args.steps // 5)):
        ctx.daq_process_batch(batch, stream=stream)
    kern_ms = ctx.kernel_times_ms()
    ctx.set_timing(False)

    # ---- pipelined: consecutive batches on two streams --------------------------------
    pipelined = None
    if not args.no_pipelined:
        # a second copy of the 16 fills (the same samples in memory of their
        # own) with a second context, output set and stream: consecutive
        # batches alternate between the two streams and overlap on the device
        log("pipelined: batches alternating over two streams")
        xd2 = distinct_copies(xd, 2)[len(xd):]
        fills2 = [daq.Fill(d, s.n_samples, threshold=s.threshold, pre=s.pre, post=s.post,
                           ped_samples=s.ped_samples) for d, s in zip(xd2, specs)]
        outs2 = [daq.alloc_out(f) for f in fills2]
        ctx2 = daq.Context(0)
        ctx2.set_graphs(graphs)  # the launch mode the tuner chose for the first context
        stream2 = torch.cuda.Stream()
        pipe = [(ctx, daq.Batch(fills, outs), stream), (ctx2, daq.Batch(fills2, outs2), stream2)]
        pipelined = None
        # overlapping batches want a smaller persistent grid: try the tuned one and 8 per CU
        for cand in sorted({sched, (sched[0], 8, sched[2], sched[3])}):
            ctx.set_schedule(*cand)
            ctx2.set_schedule(*cand)
            for i in range(4):
                c, b, st = pipe[i % 2]
                c.daq_process_batch(b, stream=st)
            torch.cuda.synchronize()
            tp0 = time.perf_counter()
            for i in range(args.steps):
                c, b, st = pipe[i % 2]
                c.daq_process_batch(b, stream=st)
            torch.cuda.synchronize()
            pipe_ms = (time.perf_counter() - tp0) * 1e3 / args.steps
            if pipelined is None or pipe_ms < pipelined["ms_per_batch"]:
                pipelined = {"streams": 2, "steps": args.steps, "ms_per_batch": round(pipe_ms, 4),
                             "gbs": round(raw_bytes / (pipe_ms * 1e-3) / 1e9, 1),
                             "pct_hbm_peak": round(100 * raw_bytes / (pipe_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 2),
                             "schedule": {"threads": cand[0], "wgs_per_cu": cand[1], "variant": cand[2],
                                          "parts": cand[3]},
                             "what": "consecutive 16-fill batches alternating over two HIP streams, each stream "
                                     "with its own context, copy of the fills and output set"}
        # the second stream's results equal the first's, element by element
        # (the same samples): islands, counts, pedestals and packed rows
        torch.cuda.synchronize()
        same = True
        for o1, o2 in zip(outs, outs2):
            n1, t1_ = int(o1.counts[0].item()), int(o1.counts[1].item())
            same = same and torch.equal(o1.counts, o2.counts) and torch.equal(o1.ped, o2.ped) \
                and torch.equal(o1.islands[:n1], o2.islands[:n1]) and torch.equal(o1.out[:, :t1_], o2.out[:, :t1_])
        pipelined["streams_agree"] = bool(same)
        ctx.set_schedule(*sched)
        ctx2.close()
        del xd2, fills2, outs2

    # ---- results of the timed steps, checked against the oracle on a sample --
    counts = [o.counts.cpu().numpy() for o in outs]
    n_isl = [int(c[0]) for c in counts]
    tot = [int(c[1]) for c in counts]
    status = [int(c[2]) & 0xFFFFFFFF for c in counts]
    assert all(s == 0 for s in status), status
    main_check = {}
    PENDING.append(("chop", main_check, (xs[0], specs[0], outs[0].host())))

    # ---- roofline of the chop launch --------------------------------------------
    alg_bytes = sum(2 * C * s.n_samples for s in specs) + sum(2 * C * t for t in tot) \
        + sum(24 * n for n in n_isl) + len(specs) * (24 + 4 * C)
    kmean = launch_ms
    achieved = alg_bytes / (kmean * 1e-3) / 1e9
    # the job's throughput: batches alternating over two streams when that
    # line ran (consecutive batches overlap on the device), else one stream
    single_gbs, single_ms = value, ms_per_step
    execution = "one batched launch per step on one HIP stream"
    if pipelined is not None:
        pms = pipelined["ms_per_batch"]
        pipelined["algorithmic_gbs"] = round(alg_bytes / (pms * 1e-3) / 1e9, 1)
        pipelined["pct_hbm_peak_algorithmic"] = round(100 * alg_bytes / (pms * 1e-3) / 1e9 / HBM_PEAK_GBS, 2)
        if pipelined["streams_agree"] and pipelined["gbs"] > single_gbs:
            value, ms_per_step = raw_bytes / (pms * 1e-3) / 1e9, pms
            execution = ("one batched launch per step, consecutive steps alternating over two HIP streams "
                         "(each with its own context, copy of the fills and output set)")
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("kernel_sha") == kernel_sha() and tr.get("fills") == len(specs):
            traffic = tr.get("bytes_per_launch")
    # the fetch floor of reading the island samples back from the raw rows
    recs = [o.islands[:n].cpu().numpy()[:, :2] for o, n in zip(outs, n_isl)]
    bases = [[x.data_ptr() + 2 * c * x.stride(0) for c in range(x.shape[0])] for x in xd]
    line_floor = island_line_bytes(recs, bases)
    copy_fetch = None
    if traffic is not None:
        copy_fetch = round(json.load(open(TRAFFIC_FILE))["kernels"].get("k_copy_pass", {}).get("fetch_bytes", 0))
    roofline = {"bound": "hbm", "achieved": round(achieved, 1) if achieved else None,
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                "traffic": traffic,
                "kernel": {5: "chop launch: k_scan_pass, k_edge_pass, k_copy_pass",
                           6: "chop launch: k_prepare, k_pipe"}.get(sched[2], "chop launch: k_prepare, k_chop")
                          + (" (one graph)" if graphs else " (plain launches)"),
                "kernel_ms_mean": round(kmean, 4),
                "kernel_launches_timed": args.steps,
                "timing": "HIP events on the launch stream at both ends of the timed region",
                "library_timed_launch_ms_mean": round(float(np.mean(kern_ms)), 4) if kern_ms else None,
                "algorithmic_bytes_per_launch": alg_bytes,
                "island_line_floor": {"bytes": line_floor, "copied_bytes": sum(2 * C * t for t in tot),
                                      "copy_pass_fetch_bytes": copy_fetch,
                                      "what": "bytes of the 128-byte lines holding island samples in the "
                                              "raw rows (the least a copy from the raw rows fetches), the "
                                              "island samples themselves, and what the copy pass fetched "
                                              "by the counter runs"}}

    # ---- plain per-fill launches (the form batching must beat) ---------------------
    plain = {}
    if not args.no_plain:
        for mode in ("fused", "twopass"):
            lat = []
            per_fill = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                        for _ in range(len(fills))]
            for _ in range(max(2, args.warmup // 2)):
                for f, o in zip(fills, outs):
                    if mode == "fused":
                        ctx.daq_chop_fill(f, o, stream)
                    else:
                        ctx.daq_find_islands(f, o, stream)
                        ctx.daq_gather_islands(f, o, stream)
            torch.cuda.synchronize()
            steps = max(3, args.steps // 4)
            tp0 = time.perf_counter()
            for _ in range(steps):
                for i, (f, o) in enumerate(zip(fills, outs)):
                    per_fill[i][0].record(stream)
                    if mode == "fused":
                        ctx.daq_chop_fill(f, o, stream)
                    else:
                        ctx.daq_find_islands(f, o, stream)
                        ctx.daq_gather_islands(f, o, stream)
                    per_fill[i][1].record(stream)
                torch.cuda.synchronize()
                lat += [a.elapsed_time(b) for a, b in per_fill]
            tp1 = time.perf_counter()
            pms = (tp1 - tp0) * 1e3 / steps
            plain[mode] = {"gbs": round(raw_bytes / (pms * 1e-3) / 1e9, 1), "ms_per_step": round(pms, 4),
                           "p50_fill_ms": round(pct(lat, 50), 4), "p99_fill_ms": round(pct(lat, 99), 4)}
            log("plain %s: %.1f GB/s" % (mode, plain[mode]["gbs"]))
        log("plain form at the single-fill shape (nominal rate)")
        plain["c0"] = plain_c0_bench(daq, synth, ctx)

    # ---- plain HBM rates for context ------------------------------------------------
    ceil = ceiling(daq)
    log("ceiling: streaming read %.0f GB/s, device copy %.0f GB/s" % (ceil["read_gbs"], ceil["copy_gbs"]))

    # ---- the Q-method on the same fills ---------------------------------------------------
    qmethod = None
    if not args.no_qmethod:
        log("Q-method on the %d fills" % len(specs))
        qmethod = q_bench(daq, ctx, xs, fills, specs, steps=max(10, args.steps // 2), warmup=3)
        log("Q-method: %.1f GB/s raw, %.0f GB/s algorithmic" % (qmethod["raw_gbs"], qmethod["roofline"]["achieved"]))

    tq = None
    if not args.no_tq:
        log("T-method and Q-method in one pass on the %d fills" % len(specs))
        tq = tq_bench(daq, ctx, xs, fills, specs, steps=max(10, args.steps // 2))
        log("T+Q: fused %.3f ms, separate %.3f ms" % (tq["fused_ms"], tq["separate_ms"]))

    ingest = None
    if not args.no_ingest:
        log("12-bit ingest of the %d fills" % len(specs))
        ingest = ingest12_bench(daq, ctx, xs, specs, steps=max(10, args.steps // 5))
        log("12-bit ingest: unpack %.0f GB/s of int16 samples" % ingest["raw_gbs"])

    compress = None
    if not args.no_compress:
        log("compression of the %d chopped fills" % len(specs))
        compress = z_bench(daq, ctx, outs, xs[0], specs[0], steps=max(10, args.steps // 2))
        log("compression: %.0f GB/s of packed samples, ratio %.2f" % (compress["packed_gbs"], compress["ratio"]))

    fig2 = None
    if not args.no_fig2:
        log("Figure 2 analog: threshold sweep, found vs true islands")
        fig2 = fig2_bench(daq, synth, ctx)
        log("Figure 2 analog: found/true %s at k = %s" % (fig2["ratio"], FIG2_KS))

    # ---- the other batch shapes: uneven batch, whole-detector stress -----------------
    others = {}
    if not args.no_uneven:
        others["uneven"] = batch_bench(daq, synth, synth.config_c2(), UNEVEN, steps=max(10, args.steps // 2),
                                      name="c2")
    if not args.no_stress:
        others["stress"] = batch_bench(daq, synth, synth.config_c4(), STRESS, steps=max(5, args.steps // 10),
                                      name="c4")
    if not args.no_served_shape:
        others["served_shape"] = batch_bench(daq, synth, [synth.config_c3_fill(s, 0) for s in range(16)], SERVED,
                                             steps=max(10, args.steps // 2), name="c3 batched")

    # ---- serving loop: Poisson arrivals with bursts, HBM-budget admission -------------
    serving = None
    if args.serve_seconds > 0:
        ps = pipelined["schedule"] if pipelined else {"threads": sched[0], "wgs_per_cu": sched[1],
                                                      "variant": sched[2], "parts": sched[3]}
        ctx.set_schedule(ps["threads"], ps["wgs_per_cu"], ps["variant"], ps["parts"])
        serving = serve_bench(daq, synth, ctx, args.serve_seconds)
        serving["schedule"] = ps
        ctx.set_schedule(*sched)

    # ---- CPU oracle: parity of every line's first fill, then its rate on a bounded sample ----
    cpu = None
    if args.cpu_seconds > 0:
        try:
            import oracle
            log("oracle checks of %d lines" % len(PENDING))
            for kind, into, payload in PENDING:
                into["parity_fill0"] = oracle_check(oracle, kind, payload)
            threads = len(os.sched_getaffinity(0))

            def one(i):
                sp = specs[i % len(specs)]
                oracle.chop(xs[i % len(specs)], n_samples=sp.n_samples, ped_samples=sp.ped_samples,
                            threshold=sp.threshold, pre=sp.pre, post=sp.post)
                return sp.raw_bytes

            # one core: whole fills in turn for a fifth of the budget
            log("CPU oracle on one core for ~%.0f s" % (args.cpu_seconds / 5))
            done1, k = 0, 0
            ts0 = time.perf_counter()
            while time.perf_counter() - ts0 < args.cpu_seconds / 5:
                done1 += one(k)
                k += 1
            single = done1 / (time.perf_counter() - ts0) / 1e9
            # every core the process may run on: one fill per thread at a time
            log("CPU oracle baseline on %d threads for ~%.0f s" % (threads, args.cpu_seconds))
            done = 0
            tc0 = time.perf_counter()
            with cf.ThreadPoolExecutor(threads) as ex:
                while time.perf_counter() - tc0 < args.cpu_seconds:
                    done += sum(ex.map(one, range(max(threads, len(specs)))))
            tc1 = time.perf_counter()
            model = cpu_model()
            cpu = {"value": round(done / (tc1 - tc0) / 1e9, 3), "unit": "GB/s", "cores": threads,
                   "kind": "oracle",
                   "sample": "the %d bench fills, each chopped whole by one thread, %d threads at a time, "
                             "repeated for %.1f s (%.2f GB raw)" % (len(specs), threads, tc1 - tc0, done / 1e9),
                   "cpu_model": model, "nproc": os.cpu_count(), "threads": threads,
                   "single_core_gbs": round(single, 3)}
            # the single-core rate on the first fills of every other timed configuration
            per = {}
            for name, (sx, ss) in ORACLE_SAMPLES.items():
                done_c, k = 0, 0
                t0c = time.perf_counter()
                while time.perf_counter() - t0c < 1.0 or k < len(sx):
                    sp = ss[k % len(ss)]
                    oracle.chop(sx[k % len(sx)], n_samples=sp.n_samples, ped_samples=sp.ped_samples,
                                threshold=sp.threshold, pre=sp.pre, post=sp.post)
                    done_c += sp.raw_bytes
                    k += 1
                per[name] = round(done_c / (time.perf_counter() - t0c) / 1e9, 3)
            cpu["single_core_gbs_by_config"] = per
        except ImportError:
            cpu = None

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "16 fills x 54 ch x 560,000 int16 samples, 3x pulse rate, "
                               "thr -200, pre 8, post 24; one batched launch per step",
                   "execution": execution,
                   "fills": len(specs), "channels": C, "samples": N, "rate": 3.0,
                   "threshold": -200, "pre": 8, "post": 24, "ped_samples": 100,
                   "schedule": {"threads": sched[0], "wgs_per_cu": sched[1], "variant": sched[2],
                                "parts": sched[3], "graphs": graphs},
                   "seeds": [s.seed for s in specs]},
        "device": device_info(),
        "host": {"cpu_model": cpu_model(), "nproc": os.cpu_count()},
        "pct_hbm_peak": round(100 * value / HBM_PEAK_GBS, 2),
        "batched": {"gbs": round(single_gbs, 1), "ms_per_step": round(single_ms, 4),
                    "pct_hbm_peak": round(100 * single_gbs / HBM_PEAK_GBS, 2),
                    "p50_fill_ms": round(pct(step_ms, 50), 4), "p99_fill_ms": round(pct(step_ms, 99), 4),
                    "what": "one stream: each launch starts when the previous one has ended"},
        "pipelined": pipelined,
        "plain": plain,
        "islands_per_fill": round(float(np.mean(n_isl)), 1),
        "islands": n_isl,
        "occupancy": round(sum(tot) / (N * len(specs)), 4),
        "parity_fill0": main_check.get("parity_fill0"),
        "roofline": roofline,
        "hbm_ceiling": ceil,
        "qmethod": qmethod,
        "tq_fused": tq,
        "ingest12": ingest,
        "compress": compress,
        "fig2_analog": fig2,
        "other_batches": others,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
