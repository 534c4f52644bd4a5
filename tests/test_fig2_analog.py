"""A Figure 2 analog on the CPU oracle (Section 3: identified islands against
the simulator's true islands at several thresholds). Truth here is the same
chop applied to the noiseless rendering of the same fill (the generator's
noise is counter-based, so dropping it leaves every pulse in place).

Checked: away from the noise (4 sigma and more below the pedestal-subtracted
baseline) the found islands match the true ones to a few per cent; within
about 2 sigma noise crossings inflate them several times over; and the marks
nest with the threshold (a lower threshold flags a subset of samples, so each
of its islands lies inside one of the higher threshold's and the packed
length does not grow). Per true pulse: every pulse deeper than 1.5 times the
threshold's depth below the baseline starts inside a found island, while
pulses shallower than half of it are caught only when they sit in another
pulse's island. No GPU: the GPU side of the same counts is checked in
tests/test_gpu_fig2.py."""
import numpy as np
import pytest

import oracle
import synth

SIGMA_SUM = 3.0 * np.sqrt(synth.CHANNELS)   # the generator's noise, summed over the crystals


def fill(index, n_samples=synth.FILL_SAMPLES):
    sp = synth.FillSpec(seed=synth.fill_seed("fig2", 0, index), n_samples=n_samples)
    return sp, synth.render(sp), synth.render(sp, noise_sigma=0.0)


def baseline(x, n):
    """Median of the pedestal-subtracted calorimeter sum (pulses at the start
    of the fill pull the pedestals low, so it sits above zero)."""
    return int(np.median(oracle.calo_sum(x, oracle.pedestals(x, n), n)))


def chop(x, n, thr):
    return oracle.chop(x, n_samples=n, ped_samples=100, threshold=thr, pre=8, post=24)


@pytest.fixture(scope="module")
def fills():
    return [fill(i) for i in range(2)]


@pytest.mark.parametrize("k", [4, 6, 10, 20])
def test_found_matches_truth_away_from_noise(fills, k):
    for sp, x, x0 in fills:
        thr = int(baseline(x, sp.n_samples) - k * SIGMA_SUM)
        found = chop(x, sp.n_samples, thr).n_islands
        truth = chop(x0, sp.n_samples, thr).n_islands
        assert truth > 700
        assert abs(found / truth - 1.0) < 0.03, (k, thr, found, truth)


def test_noise_crossings_inflate_the_count(fills):
    for sp, x, x0 in fills:
        thr = int(baseline(x, sp.n_samples) - 2 * SIGMA_SUM)
        found = chop(x, sp.n_samples, thr).n_islands
        truth = chop(x0, sp.n_samples, thr).n_islands
        assert found > 3 * truth, (thr, found, truth)


def test_islands_nest_with_the_threshold():
    sp, x, _ = fill(5, n_samples=120_000)
    b = baseline(x, sp.n_samples)
    prev = None
    for k in [0.5, 1, 2, 3, 5, 8, 15, 30]:
        r = chop(x, sp.n_samples, int(b - k * SIGMA_SUM))
        if prev is not None:
            assert r.total_len <= prev.total_len
            # every island of the lower threshold lies inside one of the higher's
            starts, stops = prev.islands[:, 0], prev.islands[:, 1]
            j = np.searchsorted(starts, r.islands[:, 0], side="right") - 1
            assert (j >= 0).all()
            assert (r.islands[:, 1] <= stops[j]).all()
        prev = r


@pytest.mark.parametrize("k", [10, 20])
def test_pulse_efficiency_by_amplitude(k):
    """Per pulse of the generator's truth list (start time, summed amplitude):
    found when its start lies inside an island."""
    for index in range(2):
        sp = synth.FillSpec(seed=synth.fill_seed("fig2", 0, index))
        x, truth = synth.render(sp, truth=True)
        depth = k * SIGMA_SUM
        r = chop(x, sp.n_samples, int(baseline(x, sp.n_samples) - depth))
        starts, stops = r.islands[:, 0], r.islands[:, 1]
        j = np.searchsorted(starts, truth["t0"], side="right") - 1
        inside = (j >= 0) & (truth["t0"] < stops[np.maximum(j, 0)])
        deep = truth["amp"] >= 1.5 * depth
        shallow = truth["amp"] < 0.5 * depth
        assert deep.sum() > 1000 and shallow.sum() > 20
        assert inside[deep].all()
        assert inside[shallow].mean() < 0.8
