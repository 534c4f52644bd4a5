"""The synthetic fill generator: determinism, ranges and the workload shape."""
import numpy as np

import synth


def test_same_seed_same_bytes_any_thread_count():
    spec = synth.FillSpec(seed=11, n_samples=50_003, rate=2.0)
    a = synth.render(spec, nthreads=1)
    b = synth.render(spec, nthreads=7)
    np.testing.assert_array_equal(a, b)
    c = synth.render(synth.FillSpec(seed=12, n_samples=50_003, rate=2.0))
    assert not np.array_equal(a, c)


def test_range_padding_and_stride():
    spec = synth.FillSpec(seed=3, n_samples=10_001, rate=10.0)
    x = synth.render(spec)
    assert x.shape == (54, 10_008) and spec.row_stride % 8 == 0
    assert x[:, :10_001].min() >= 0 and x[:, :10_001].max() <= 4095
    assert (x[:, 10_001:] == 0).all()


def test_pedestal_levels_and_noise():
    x = synth.render(synth.FillSpec(seed=21, n_samples=200_000, rate=0.0))
    tail = x[:, 100_000:].astype(np.float64)
    means = tail.mean(1)
    assert (means > 1699).all() and (means < 1901).all()
    sd = tail.std(1)
    assert (np.abs(sd - 3.0) < 0.15).all()


def test_pulse_count_and_time_profile():
    counts = []
    for i in range(6):
        _, tr = synth.render(synth.FillSpec(seed=100 + i), truth=True)
        counts.append(len(tr))
        assert (np.diff(tr["t0"]) >= 0).all() and tr["t0"].max() < 560_000
        assert (tr["amp"] >= 50).all() and (tr["amp"] <= 3000).all()
        assert ((tr["n_cry"] >= 1) & (tr["n_cry"] <= 4)).all()
        fr = tr["frac"].copy()
        for k in range(4):
            fr[tr["n_cry"] <= k, k] = 0
        np.testing.assert_allclose(fr.sum(1), 1.0, rtol=1e-12)
    # about 2000 pulses per fill at 1x rate (Poisson: sd ~ 45)
    assert 1850 < np.mean(counts) < 2150
    # the rate decays as exp(-t / 64.4 us): the first tau holds ~63 % of pulses
    _, tr = synth.render(synth.FillSpec(seed=7, rate=5.0), truth=True)
    frac = (tr["t0"] < synth.TAU_SAMPLES).mean()
    assert 0.60 < frac < 0.66


def test_clusters_are_connected_neighbours():
    _, tr = synth.render(synth.FillSpec(seed=8, n_samples=100_000, rate=2.0), truth=True)
    for p in tr[:300]:
        cells = [(c // 9, c % 9) for c in p["cry"][:p["n_cry"]]]
        assert len(set(cells)) == len(cells)
        seen = {cells[0]}
        frontier = [cells[0]]
        while frontier:
            r, c = frontier.pop()
            for q in ((r + 1, c), (r - 1, c), (r, c + 1), (r, c - 1)):
                if q in cells and q not in seen:
                    seen.add(q)
                    frontier.append(q)
        assert len(seen) == len(cells)


def test_config_recipes():
    assert len(synth.config_c1()) == 16 and all(s.rate == 3.0 for s in synth.config_c1())
    c2 = synth.config_c2()
    assert len(c2) == 24
    for s in c2:
        assert 100_000 <= s.n_samples <= 560_000 and 0.5 <= s.rate <= 4.0
        assert -400 <= s.threshold <= -150 and 4 <= s.pre <= 16 and 16 <= s.post <= 48
    c4 = synth.config_c4()
    assert len(c4) == 96 and all(s.threshold == -100 and s.post == 48 for s in c4)
    seeds = [s.seed for s in c4]
    assert len(set(seeds)) == len(seeds)
