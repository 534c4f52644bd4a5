"""Pins of the CPU oracle against things other than itself (CPU only).

* hand-derived golden fixtures (tests/golden/, each with its citation);
* a brute-force restatement from the window definition (tests/brute.py) on
  thousands of random tiny fills;
* numpy's own integer sum for the calorimeter sum;
* closed forms: one pulse, no crossing, touching / one-sample-gap windows,
  all below threshold, clipping at both ends, S == thr, pre = post = 0,
  constant channels, the round-half-up pedestal;
* invariants on full-size synthetic fills.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import brute  # noqa: E402
import golden_io  # noqa: E402
import oracle  # noqa: E402
import synth  # noqa: E402


def max_islands(N, pre, post):
    # islands hold at least one flagged sample each and flagged samples of
    # different islands are at least pre + post + 2 apart
    return 0 if N <= 0 else (N - 1) // (pre + post + 2) + 1


# ---------------------------------------------------------------- golden ----

@pytest.mark.parametrize("path", golden_io.fixture_files(), ids=os.path.basename)
def test_golden_fixture(path):
    g = golden_io.load(path)
    r = oracle.chop(g["x"], ped_samples=g["ped_samples"], threshold=g["threshold"],
                    pre=g["pre"], post=g["post"])
    np.testing.assert_array_equal(r.ped, g["ped"])
    np.testing.assert_array_equal(r.islands, g["islands"])
    assert r.n_islands == len(g["islands"])
    assert r.total_len == g["total_len"]
    np.testing.assert_array_equal(r.out, g["out"])


@pytest.mark.parametrize("path", golden_io.fixture_files(), ids=os.path.basename)
def test_golden_fixture_brute(path):
    # the brute force agrees with the hand-derived values too
    g = golden_io.load(path)
    ped, isl, total, out, *_ = brute.chop(g["x"].tolist(), g["samples"], g["ped_samples"],
                                          g["threshold"], g["pre"], g["post"])
    assert ped == g["ped"].tolist()
    assert [list(i) for i in isl] == g["islands"].tolist()
    assert total == g["total_len"]
    assert out == g["out"].tolist()


# ----------------------------------------------------------- brute force ----

def _random_case(rng):
    C = int(rng.integers(1, 7))
    N = int(rng.integers(0, 160))
    stride = N + int(rng.integers(0, 5))
    kind = rng.integers(0, 3)
    if kind == 0:      # arbitrary int16 values, including negatives
        x = rng.integers(-300, 300, size=(C, stride)).astype(np.int16)
    elif kind == 1:    # baseline plus sparse dips (pulse-like)
        x = (rng.integers(95, 106, size=(C, stride))).astype(np.int16)
        for _ in range(int(rng.integers(0, 6))):
            t = int(rng.integers(0, max(stride, 1)))
            x[:, t:t + int(rng.integers(1, 4))] -= rng.integers(0, 40, size=(C, 1)).astype(np.int16)
    else:              # extreme int16 values
        x = rng.choice(np.array([-32768, -1, 0, 1, 32767], np.int16), size=(C, stride))
    Np = int(rng.integers(1, 120))
    pre = int(rng.integers(0, 13))
    post = int(rng.integers(0, 13))
    ped = [brute.pedestal(list(r[:N]), Np) for r in x]
    S = x[:, :N].astype(np.int64).sum(0) - sum(ped) if N else np.zeros(0, np.int64)
    if N and rng.random() < 0.8:
        thr = int(rng.choice(S)) + int(rng.integers(-1, 2))   # thresholds on data values
    else:
        thr = int(rng.integers(-500, 500))
    return x, N, Np, thr, pre, post


def test_oracle_matches_brute_force_random():
    rng = np.random.default_rng(1234)
    for case in range(10000):
        x, N, Np, thr, pre, post = _random_case(rng)
        r = oracle.chop(x, n_samples=N, ped_samples=Np, threshold=thr, pre=pre, post=post)
        ped, isl, total, out, S, F, M = brute.chop(x.tolist(), N, Np, thr, pre, post)
        ctx = f"case {case}: C={x.shape[0]} N={N} Np={Np} thr={thr} pre={pre} post={post}"
        assert r.ped.tolist() == ped, ctx
        assert r.islands.tolist() == [list(i) for i in isl], ctx
        assert r.n_islands == len(isl) and r.total_len == total, ctx
        assert r.out.tolist() == out, ctx
        assert r.n_islands <= max_islands(N, pre, post), ctx


def test_step_functions_match_brute_force():
    rng = np.random.default_rng(99)
    for _ in range(300):
        x, N, Np, thr, pre, post = _random_case(rng)
        ped, isl, total, out, S, F, M = brute.chop(x.tolist(), N, Np, thr, pre, post)
        p = oracle.pedestals(x, n_samples=N, ped_samples=Np)
        assert p.tolist() == ped
        s = oracle.calo_sum(x, p, n_samples=N)
        assert s.tolist() == S
        f = oracle.threshold(s, thr)
        assert f.astype(bool).tolist() == F
        m = oracle.dilate(f, pre, post)
        assert m.astype(bool).tolist() == M
        rec, tl, n = oracle.islands(m)
        assert rec.tolist() == [list(i) for i in isl] and tl == total


# ----------------------------------------------------------- library sum ----

def test_calo_sum_equals_numpy_sum():
    spec = synth.FillSpec(seed=5, n_samples=20_000, rate=3.0)
    x = synth.render(spec)
    ped = oracle.pedestals(x, n_samples=spec.n_samples)
    S = oracle.calo_sum(x, ped, n_samples=spec.n_samples)
    ref = x[:, :spec.n_samples].astype(np.int64).sum(axis=0) - ped.astype(np.int64).sum()
    np.testing.assert_array_equal(S, ref)


def test_pedestal_is_rounded_mean():
    # exact half-up rounding of the mean of the first Np samples, against
    # numpy's float mean on values where float rounding is exact
    rng = np.random.default_rng(7)
    x = rng.integers(-2000, 4096, size=(54, 400)).astype(np.int16)
    for Np in (1, 2, 3, 4, 7, 100, 400, 1000):
        n = min(Np, 400)
        ped = oracle.pedestals(x, ped_samples=Np)
        ref = np.floor(x[:, :n].astype(np.float64).sum(1) / n + 0.5).astype(np.int32)
        np.testing.assert_array_equal(ped, ref)


@pytest.mark.parametrize("vals,expect", [
    ([1, 1, 1, 2], 1),      # 1.25
    ([1, 2, 2, 2], 2),      # 1.75
    ([1, 1, 2, 2], 2),      # 1.5 rounds up
    ([-1, -1, -2, -2], -1), # -1.5 rounds up
    ([-1, -2, -2, -2], -2), # -1.75
    ([0, 0, 0, 1], 0),      # 0.25
    ([0, 1, 1, 0], 1),      # 0.5
    ([0, -1, -1, 0], 0),    # -0.5
])
def test_pedestal_half_up_closed_form(vals, expect):
    x = np.array([vals + [0] * 6], np.int16)
    assert oracle.pedestals(x, ped_samples=4).tolist() == [expect]


def test_pedestal_short_fill_and_empty():
    x = np.array([[3, 4, 100, 100]], np.int16)
    assert oracle.pedestals(x, n_samples=2, ped_samples=100).tolist() == [4]  # 3.5 -> 4
    assert oracle.pedestals(x, n_samples=0, ped_samples=100).tolist() == [0]


# ----------------------------------------------------------- closed form ----

def _flat(C, N, level=1000):
    return np.full((C, N), level, np.int16)


@pytest.mark.parametrize("a,b", [(40, 40), (40, 55), (0, 3), (95, 99), (0, 30)])
@pytest.mark.parametrize("pre,post", [(0, 0), (8, 24), (3, 1), (50, 50)])
def test_single_run_gives_known_island(a, b, pre, post):
    # a dip of -500 on one channel over [a, b]; the expected pedestals come
    # from exact rational rounding, independent of the oracle
    N = 100
    x = _flat(3, N)
    x[1, a:b + 1] -= 500
    Np = 100
    ped = [brute.pedestal(list(r), Np) for r in x.tolist()]
    S = x.astype(np.int64).sum(0) - sum(ped)
    flagged = np.nonzero(S < -200)[0]
    assert flagged.min() == a and flagged.max() == b          # the dip is the crossing run
    r = oracle.chop(x, ped_samples=Np, threshold=-200, pre=pre, post=post)
    assert r.ped.tolist() == ped
    assert r.islands.tolist() == [[max(0, a - pre), min(N - 1, b + post) + 1, 0]]


def test_no_crossing_zero_islands():
    x = _flat(54, 1000)
    r = oracle.chop(x, threshold=-1)
    assert r.n_islands == 0 and r.total_len == 0 and len(r.islands) == 0


@pytest.mark.parametrize("pre,post", [(8, 24), (0, 0), (1, 0), (0, 1), (5, 7)])
def test_touching_windows_merge_and_one_gap_splits(pre, post):
    N = 300
    for gap, expect in ((pre + post + 1, 1), (pre + post + 2, 2)):
        x = _flat(2, N)
        a1 = 100
        a2 = a1 + gap
        x[0, a1] -= 300
        x[0, a2] -= 300
        r = oracle.chop(x, ped_samples=10, threshold=-100, pre=pre, post=post)
        assert r.n_islands == expect, (gap, r.islands)
        if expect == 1:
            assert r.islands.tolist() == [[a1 - pre, a2 + post + 1, 0]]
        else:
            assert r.islands.tolist() == [[a1 - pre, a1 + post + 1, 0],
                                          [a2 - pre, a2 + post + 1, pre + post + 1]]
            assert r.islands[1, 0] - r.islands[0, 1] == 1


def test_all_below_threshold_one_island():
    x = _flat(4, 777)
    r = oracle.chop(x, threshold=1)    # S == 0 < 1 everywhere
    assert r.islands.tolist() == [[0, 777, 0]] and r.total_len == 777


def test_equal_to_threshold_is_not_a_crossing():
    x = _flat(2, 200)
    x[0, 120] -= 50
    r = oracle.chop(x, threshold=-50)
    assert r.n_islands == 0
    r = oracle.chop(x, threshold=-49)
    assert r.n_islands == 1


def test_crossing_at_both_ends_is_clipped():
    N = 500
    x = _flat(2, N)
    x[0, N - 1] -= 400              # S[N-1] = -400, pedestals untouched
    r = oracle.chop(x, ped_samples=100, threshold=-100, pre=8, post=24)
    assert r.islands.tolist() == [[N - 1 - 8, N, 0]]
    x = _flat(2, N)
    x[0, 0] -= 400                  # ped0 = 996: S[0] = -396, S[t > 0] = +4
    r = oracle.chop(x, ped_samples=100, threshold=-100, pre=8, post=24)
    assert r.ped.tolist() == [996, 1000]
    assert r.islands.tolist() == [[0, 25, 0]]


def test_pre_post_zero_islands_are_flag_runs():
    rng = np.random.default_rng(3)
    x = rng.integers(990, 1010, size=(3, 5000)).astype(np.int16)
    r = oracle.chop(x, threshold=-20, pre=0, post=0)
    S = x.astype(np.int64).sum(0) - r.ped.sum()
    F = (S < -20).astype(np.int8)
    d = np.diff(np.concatenate([[0], F, [0]]))
    starts, stops = np.nonzero(d == 1)[0], np.nonzero(d == -1)[0]
    assert r.islands[:, 0].tolist() == starts.tolist()
    assert r.islands[:, 1].tolist() == stops.tolist()


def test_constant_channels_have_no_island():
    rng = np.random.default_rng(4)
    levels = rng.integers(0, 4096, size=54)
    x = np.repeat(levels[:, None], 3000, axis=1).astype(np.int16)
    for thr in (0, -1, -200):
        assert oracle.chop(x, threshold=thr).n_islands == 0
    assert oracle.chop(x, threshold=1).n_islands == 1


def test_capacity_truncates_records_but_counts_all():
    x = _flat(1, 1000)
    for t in range(10, 1000, 100):
        x[0, t] -= 200
    full = oracle.chop(x, threshold=-100, pre=2, post=2)
    part = oracle.chop(x, threshold=-100, pre=2, post=2, capacity=3)
    assert full.n_islands == 10 and part.n_islands == 10
    assert part.islands.tolist() == full.islands[:3].tolist()
    assert part.total_len == full.total_len


def test_max_islands_bound_is_reached():
    # dips every pre + post + 2 samples from t = 0 reach the bound exactly:
    # with Np = 1 the pedestal is the dip level, so S = 0 at dips, +300 elsewhere
    for pre, post, N in ((0, 0, 50), (8, 24, 1000), (3, 5, 97), (2, 2, 6)):
        x = _flat(1, N)
        x[0, 0:N:pre + post + 2] -= 300
        r = oracle.chop(x, ped_samples=1, threshold=1, pre=pre, post=post)
        assert r.n_islands == max_islands(N, pre, post) == len(range(0, N, pre + post + 2))


# ------------------------------------------------------------ invariants ----

@pytest.mark.parametrize("spec", [synth.config_c0()[0], synth.config_c1(1)[0],
                                  synth.config_c4(1, 1)[0], synth.config_c2()[3]],
                         ids=["c0", "c1", "c4", "c2s3"])
def test_invariants_on_synthetic_fill(spec):
    x = synth.render(spec)
    N = spec.n_samples
    r = oracle.chop(x, n_samples=N, threshold=spec.threshold, pre=spec.pre, post=spec.post)
    isl = r.islands
    S = x[:, :N].astype(np.int64).sum(0) - r.ped.astype(np.int64).sum()
    F = S < spec.threshold
    assert r.n_islands == len(isl) > 0
    lengths = isl[:, 1] - isl[:, 0]
    assert (lengths > 0).all()
    assert (isl[1:, 0] > isl[:-1, 1]).all()                      # sorted, gap >= 1
    assert (isl[:, 2] == np.concatenate([[0], np.cumsum(lengths)[:-1]])).all()
    assert lengths.sum() == r.total_len
    inside = np.zeros(N, bool)
    for s, e, _ in isl:
        inside[s:e] = True
        assert F[s:e].any()                                       # each holds a crossing
    assert inside[F].all()                                        # every crossing covered
    interior = (isl[:, 0] > 0) & (isl[:, 1] < N)
    assert (lengths[interior] >= spec.pre + spec.post + 1).all()
    assert r.n_islands <= max_islands(N, spec.pre, spec.post)
    for s, e, o in isl[:: max(1, len(isl) // 50)]:
        np.testing.assert_array_equal(r.out[:, o:o + e - s], x[:, s:e])
    # the island edges sit exactly pre before a crossing and post after one
    for s, e, _ in isl[:: max(1, len(isl) // 50)]:
        if s > 0:
            assert F[s + spec.pre] and not F[max(0, s - 1 - spec.post):s + spec.pre].any()
        if e < N:
            assert F[e - 1 - spec.post] and not F[e - spec.post:min(N, e + spec.pre + 1)].any()
