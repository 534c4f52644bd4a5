"""The serving loop's host code under AddressSanitizer and
UndefinedBehaviorSanitizer: tests/native/server_stress (built by
__graft_entry__.build() against a copy of the library whose host code is
instrumented) drives a server from three submitter threads and a poller for
three seconds, with a budget that refuses fills and a batch time-out switched
to 1 us and back while batches run; every completion must match the same
fill's first result, and the sanitizers must report nothing."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU machines
    pytest.skip("no GPU", allow_module_level=True)

from paper_1611_04959_amd import build as B  # noqa: E402


def test_server_stress_under_sanitizers():
    if not os.path.exists(B.SAN_STRESS):
        pytest.skip("tests/native/sanitized is not built (run __graft_entry__.build())")
    env = dict(os.environ)
    # leaks of the HIP runtime at exit are not ours; errors stop the program
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    # the library's default schedule: with fill groups forced (extra streams
    # per context) ASan's allocator has failed a check inside the HIP
    # runtime's own teardown at exit, after the program had finished
    env.pop("DAQ_SCHEDULE", None)
    print("server_stress 3 s under ASan + UBSan", flush=True)
    r = subprocess.run([B.SAN_STRESS, "3"], capture_output=True, text=True, timeout=90, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    fields = dict(zip(r.stdout.split()[0::2], r.stdout.split()[1::2]))
    assert int(fields["completed"]) == int(fields["submitted"]) > 1000
    assert int(fields["mismatched"]) == 0 and int(fields["errors"]) == 0
    assert int(fields["refused"]) > 0 and int(fields["timed_out"]) > 0


def test_server_stress_with_logging_under_sanitizers():
    """The same stress with DAQ_LOG=2: the diagnostic lines of several
    threads (batches given up by the watchdog, deadtime periods, creation and
    shutdown) are written under the sanitizers too, each line whole."""
    if not os.path.exists(B.SAN_STRESS):
        pytest.skip("tests/native/sanitized is not built (run __graft_entry__.build())")
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["DAQ_LOG"] = "2"
    env.pop("DAQ_SCHEDULE", None)
    print("server_stress 1 s under ASan + UBSan with DAQ_LOG=2", flush=True)
    r = subprocess.run([B.SAN_STRESS, "1"], capture_output=True, text=True, timeout=90, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, r.stderr[-4000:]
    lines = [ln for ln in r.stderr.splitlines() if "[daq]" in ln]
    assert all(ln.startswith("[daq] ") for ln in lines), [ln for ln in lines if not ln.startswith("[daq] ")][:5]
    assert any("server on device 0: 3 workers" in ln for ln in lines)
    assert any("server shut down:" in ln for ln in lines)
    assert any("outlived" in ln for ln in lines)  # the 1 us time-out gave up on batches
    assert any("deadtime begins" in ln for ln in lines)
