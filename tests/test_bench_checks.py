"""The bench's parity report (bench.oracle_check), on the CPU: for every kind
of line it accepts results equal to the oracle's and rejects a result with one
element changed, so a parity_fill0 of true in the bench line means what it
says."""
import dataclasses
import importlib.util
import os

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.fixture(scope="module")
def fill():
    sp = synth.FillSpec(seed=synth.fill_seed("bench-check", 0, 0), n_samples=20_003, rate=3.0)
    return sp, synth.render(sp)


def _chop(x, sp):
    return oracle.chop(x, n_samples=sp.n_samples, ped_samples=sp.ped_samples, threshold=sp.threshold,
                       pre=sp.pre, post=sp.post)


def _host(ref):
    return (ref.islands.copy(), ref.n_islands, ref.total_len, 0, ref.ped.copy(), ref.out.copy())


def test_chop_line(bench, fill):
    sp, x = fill
    ref = _chop(x, sp)
    assert ref.n_islands > 5
    assert bench.oracle_check(oracle, "chop", (x, sp, _host(ref)))
    isl, n, total, st, ped, out = _host(ref)
    out[3, 7] += 1
    assert not bench.oracle_check(oracle, "chop", (x, sp, (isl, n, total, st, ped, out)))
    assert not bench.oracle_check(oracle, "chop", (x, sp, (isl, n, total, 1, ped, ref.out)))


def test_qmethod_and_fused_lines(bench, fill):
    sp, x = fill
    N, k = sp.n_samples, 3
    ped, Q = oracle.qmethod(x, N, ped_samples=sp.ped_samples)
    acc = ((k * (x[:, :N].astype(np.int64) - ped[:, None])) % 2**32).astype(np.uint32).view(np.int32)
    assert bench.oracle_check(oracle, "qmethod", (x, sp, k, Q.copy(), acc))
    bad = acc.copy()
    bad[0, 0] += 1
    assert not bench.oracle_check(oracle, "qmethod", (x, sp, k, Q.copy(), bad))
    assert not bench.oracle_check(oracle, "qmethod", (x, sp, k + 1, Q.copy(), acc))
    ref = _chop(x, sp)
    assert bench.oracle_check(oracle, "tq", (x, sp, k, _host(ref), Q.copy(), acc))
    Qb = Q.copy()
    Qb[-1] += 1
    assert not bench.oracle_check(oracle, "tq", (x, sp, k, _host(ref), Qb, acc))


def test_compress_and_fig2_lines(bench, fill):
    sp, x = fill
    ref = _chop(x, sp)
    hdr, words = oracle.z_compress(ref.out, ref.total_len)
    assert bench.oracle_check(oracle, "compress", (x, sp, hdr.copy(), words.copy()))
    w2 = words.copy()
    w2[len(w2) // 2] ^= 4
    assert not bench.oracle_check(oracle, "compress", (x, sp, hdr.copy(), w2))
    x0 = synth.render(sp, noise_sigma=0.0)
    thrs = [-150, -300]
    found = [_chop(x, dataclasses.replace(sp, threshold=t)).n_islands for t in thrs]
    truth = [_chop(x0, dataclasses.replace(sp, threshold=t)).n_islands for t in thrs]
    assert bench.oracle_check(oracle, "fig2", (x, x0, sp, thrs, found, truth))
    assert not bench.oracle_check(oracle, "fig2", (x, x0, sp, thrs, [found[0] + 1, found[1]], truth))
    with pytest.raises(ValueError):
        bench.oracle_check(oracle, "unknown", None)


def test_traffic_hash_follows_code_not_comments(tmp_path, monkeypatch):
    """The traffic counts stay attached to the kernel code they were taken
    for: a comment or spacing edit keeps the hash, any code edit changes it
    (the bench then reports the traffic as unknown)."""
    from paper_1611_04959_amd import traffic
    src = tmp_path / "k.hip"
    src.write_text("// scan\nint f(int x) {\n  return x + 1;  /* one */\n}\n")
    monkeypatch.setattr(traffic, "KERNEL_SOURCES", [str(src)])
    h0 = traffic.kernel_sha()
    src.write_text("// the scan pass\nint f(int x) {   return x + 1; /* one,\n two */ }\n")
    assert traffic.kernel_sha() == h0
    src.write_text("// scan\nint f(int x) {\n  return x + 2;  /* one */\n}\n")
    assert traffic.kernel_sha() != h0


def test_arrivals_rate_and_bursts(bench):
    """The serving workload's arrivals: a Poisson process whose long-run mean
    is the requested rate, 5 times denser inside the 80 ms bursts that take a
    tenth of the time, and sorted."""
    rng = np.random.default_rng(11)
    rate, seconds = 2000.0, 40.0
    t = np.array(bench.arrivals(rate, seconds, rng))
    assert np.all(np.diff(t) >= 0) and t[0] >= 0 and t[-1] < seconds
    assert abs(len(t) / seconds - rate) < 0.03 * rate
    in_burst = (t % 0.8) < 0.08
    dense = in_burst.sum() / (0.1 * seconds)
    sparse = (~in_burst).sum() / (0.9 * seconds)
    assert 4.5 < dense / sparse < 5.5


def test_island_line_bytes_against_brute_force(bench):
    rng = np.random.default_rng(3)
    records, bases, want = [], [], 0
    for _ in range(5):
        n = int(rng.integers(0, 12))
        cuts = np.sort(rng.choice(np.arange(1, 4000), size=2 * n, replace=False))
        rec = cuts.reshape(-1, 2)  # disjoint [start, stop), increasing
        row = [int(rng.integers(0, 1 << 20)) * 2 for _ in range(3)]
        records.append(rec)
        bases.append(row)
        for b in row:
            lines = {(b + 2 * t + k) // 128 for s, e in rec for t in range(s, e) for k in (0, 1)}
            want += 128 * len(lines)
    assert bench.island_line_bytes(records, bases) == want
    # two islands in one line count it once; one sample straddling nothing
    assert bench.island_line_bytes([np.array([[0, 10], [20, 30]])], [[0]]) == 128
    assert bench.island_line_bytes([np.array([[63, 65]])], [[0]]) == 256
