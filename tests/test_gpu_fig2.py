"""GPU side of the Figure 2 analog: one fill chopped at thresholds from 1 to
20 sigma below its baseline, noisy and noiseless renderings in one batched
launch (all entries of a threshold sweep read the same raw rows), every
island table and packed row equal to the oracle's, and the found/true ratio
near 1 away from the noise."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU machines
    pytest.skip("no GPU", allow_module_level=True)

import paper_1611_04959_amd as daq  # noqa: E402
from gpu_util import assert_same, log  # noqa: E402

SIGMA_SUM = 3.0 * np.sqrt(synth.CHANNELS)
KS = [1, 2, 4, 10, 20]


def test_threshold_sweep_matches_oracle():
    sp = synth.FillSpec(seed=synth.fill_seed("fig2", 0, 0))
    N = sp.n_samples
    x = synth.render(sp)
    x0 = synth.render(sp, noise_sigma=0.0)
    b = int(np.median(oracle.calo_sum(x, oracle.pedestals(x, N), N)))
    thrs = [int(b - k * SIGMA_SUM) for k in KS]
    xd, x0d = synth.to_device([x, x0])
    fills = [daq.Fill(d, N, threshold=t, pre=8, post=24, ped_samples=100) for d in (xd, x0d) for t in thrs]
    outs = [daq.alloc_out(f) for f in fills]
    with daq.Context(0) as ctx:
        log("fig2 sweep: %d fills sharing two raw buffers" % len(fills))
        ctx.daq_process_batch(fills, outs)
        torch.cuda.synchronize()
    refs = [oracle.chop(h, n_samples=N, ped_samples=100, threshold=t, pre=8, post=24)
            for h in (x, x0) for t in thrs]
    for i, (o, r) in enumerate(zip(outs, refs)):
        assert_same(o, r, ctx="entry %d (thr %d)" % (i, fills[i].threshold))
    found = [int(o.counts[0].item()) for o in outs[:len(KS)]]
    truth = [int(o.counts[0].item()) for o in outs[len(KS):]]
    log("k, found, truth: %s" % list(zip(KS, found, truth)))
    for k, f, t in zip(KS, found, truth):
        if k >= 4:
            assert abs(f / t - 1.0) < 0.03
