"""The library's environment variables on the GPU: DAQ_SCHEDULE fixes a new
context's schedule and graph mode (the tuner then keeps it, and results still
match the oracle), a malformed or refused value fails the context's creation
with a reason on stderr, and DAQ_LOG=2 reports the context, the schedule's
origin, the tuner's decision and scratch growth while DAQ_LOG unset prints
nothing. Each case runs in a child process, since the library reads DAQ_LOG
once per process."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU machines
    pytest.skip("no GPU", allow_module_level=True)

from gpu_util import log  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.join(ROOT, "tests")

# Six random 54-channel fills of 40,000 samples (several tiles, a ragged
# tail), chopped once under the context's schedule, then through the tuner
# and once more; every result is compared with the oracle.
CHILD = r"""
import json, sys
import numpy as np
import torch
import paper_1611_04959_amd as daq
from gpu_util import assert_same, dev, make_fill, oracle_many, pad_stride, run

rng = np.random.default_rng(11)
C, N = 54, 40_000
xs = []
for _ in range(6):
    x = rng.integers(1750, 1850, (C, N)).astype(np.int16)
    for t0 in rng.integers(0, N - 40, 30):
        x[:, t0:t0 + 25] -= 300
    xs.append(pad_stride(x))
p = {"threshold": -2000, "pre": 8, "post": 24, "ped_samples": 100}
refs = oracle_many(xs, [N] * 6, [p] * 6)
ctx = daq.Context(0)
s = ctx.get_schedule()
out = {"schedule": [s.threads, s.wgs_per_cu, s.variant, s.parts], "graphs": ctx.get_graphs()}
fills = [make_fill(dev(x), N, p) for x in xs]
outs = [daq.alloc_out(f) for f in fills]
run(ctx, "batch", fills, outs)
for i, (o, r) in enumerate(zip(outs, refs)):
    assert_same(o, r, ctx="fill %d before tuning" % i)
best = ctx.daq_autotune(fills, outs)
out["best"] = [best.threads, best.wgs_per_cu, best.variant, best.parts]
run(ctx, "batch", fills, outs)
for i, (o, r) in enumerate(zip(outs, refs)):
    assert_same(o, r, ctx="fill %d after tuning" % i)
out["islands"] = int(sum(r.n_islands for r in refs))
ctx.close()
print(json.dumps(out), flush=True)
"""


def _child(env_extra, code=CHILD, timeout=240):
    env = {k: v for k, v in os.environ.items() if k not in ("DAQ_LOG", "DAQ_SCHEDULE")}
    env.update(env_extra)
    env["PYTHONPATH"] = os.pathsep.join([ROOT, TESTS, env.get("PYTHONPATH", "")])
    log("child with %s" % env_extra)
    return subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=timeout, env=env)


def _daq_lines(stderr):
    return [ln for ln in stderr.splitlines() if ln.startswith("[daq] ")]


def test_schedule_from_env_is_kept_and_logged():
    r = _child({"DAQ_SCHEDULE": "256,16,5,2,0", "DAQ_LOG": "2"})
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    res = json.loads(r.stdout.strip().splitlines()[-1])
    assert res["schedule"] == [256, 16, 5, 2]
    assert res["graphs"] is False
    assert res["best"] == [256, 16, 5, 2]  # the tuner keeps a pinned schedule
    assert res["islands"] > 0
    lines = _daq_lines(r.stderr)
    assert any("context on device 0" in ln and "256/16/5/2 (DAQ_SCHEDULE)" in ln for ln in lines), lines
    assert any("fixed by DAQ_SCHEDULE, not tuned" in ln for ln in lines), lines
    assert any("scratch of stream" in ln for ln in lines), lines
    assert not any("median" in ln for ln in lines), lines  # nothing was timed


def test_tuner_decisions_logged_and_silent_by_default():
    r = _child({"DAQ_LOG": "2"})
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    res = json.loads(r.stdout.strip().splitlines()[-1])
    lines = _daq_lines(r.stderr)
    timed = [ln for ln in lines if "autotune: schedule" in ln and "median" in ln]
    kept = [ln for ln in lines if "autotune: kept" in ln]
    assert len(timed) >= 5 and len(kept) == 1, lines
    assert "kept %d/%d/%d/%d" % tuple(res["best"]) in kept[0]
    assert any("graphs captured" in ln for ln in lines), lines
    # the same work with DAQ_LOG unset writes no diagnostic line
    q = _child({})
    assert q.returncode == 0, q.stdout[-2000:] + q.stderr[-4000:]
    assert _daq_lines(q.stderr) == []


@pytest.mark.parametrize("value", ["512,8,5", "512,8,5,0,2", "128,8,5,0", "512,8,5,0x", "256,99,5,0"])
def test_refused_schedule_fails_context_creation(value):
    code = ("import paper_1611_04959_amd as daq\n"
            "try:\n    daq.Context(0)\nexcept daq.DaqError as e:\n    print('code', e.code)\n"
            "else:\n    print('created')\n")
    r = _child({"DAQ_SCHEDULE": value}, code=code, timeout=120)
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.strip().splitlines()[-1] == "code -1"
    assert any('DAQ_SCHEDULE="%s" refused' % value in ln for ln in _daq_lines(r.stderr)), r.stderr[-2000:]
