"""The C ABI library loads and exports every call include/daq.h declares
(CPU only: nothing here launches GPU work)."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

import paper_1611_04959_amd as daq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "daq.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(daq_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("daq_find_islands", "daq_gather_islands", "daq_chop_fill", "daq_process_batch",
                     "daq_max_islands", "daq_ctx_create", "daq_ctx_destroy", "daq_autotune"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = daq.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", daq.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (daq_[a-z_0-9]+)$", out, flags=re.M))
    assert set(declared_functions()) <= exported


def test_library_is_built_for_gfx950_only():
    # the offload bundle names each device target it carries
    blob = open(daq.LIB_PATH, "rb").read()
    targets = set(re.findall(rb"hipv4-amdgcn-amd-amdhsa--(gfx[0-9a-z]+)", blob))
    assert targets == {b"gfx950"}


def test_version_and_strerror():
    assert "gfx950" in daq.version()
    lib = daq.load_library()
    for code in range(-8, 1):
        assert lib.daq_strerror(code)


def test_max_islands_bound():
    for N, pre, post in ((0, 8, 24), (1, 8, 24), (560_000, 8, 24), (100, 0, 0), (7, 1, 1)):
        expect = 0 if N <= 0 else (N - 1) // (pre + post + 2) + 1
        assert daq.daq_max_islands(N, pre, post) == expect
    assert daq.daq_max_islands(10, -1, 0) == -1
    # the configuration bound quoted for the plain workload
    assert daq.daq_max_islands(560_000, 8, 24) == 16_471


def test_null_context_is_rejected_without_touching_a_gpu():
    lib = daq.load_library()
    f = daq.daq_fill(0, 0, 0, 1, 100, -200, 8, 24, 0)
    rc = lib.daq_find_islands(None, ctypes.byref(f), None, 0, None, None, None)
    assert rc == daq.DAQ_EINVAL
    rc = lib.daq_process_batch(None, None, None, 0, None)
    assert rc == daq.DAQ_EINVAL


def test_struct_layouts_match_header():
    assert ctypes.sizeof(daq.daq_fill) == 48
    assert ctypes.sizeof(daq.daq_fill_out) == 48
    assert ctypes.sizeof(daq.daq_schedule) == 16


def test_server_slot_bytes_layout():
    lib = daq.load_library()
    up = lambda n: (n + 255) // 256 * 256
    b = ctypes.c_uint64(0)
    for C, N, stride, pre, post, flags in ((54, 560_000, 560_000, 8, 24, 0), (54, 560_000, 560_000, 8, 24, 1),
                                           (3, 1001, 1008, 0, 0, 0), (1, 0, 0, 4, 4, 0)):
        f = daq.daq_fill(0x1000 if N else 0, N, stride, C, 100, -200, pre, post, 0)
        assert lib.daq_server_slot_bytes(ctypes.byref(f), flags, ctypes.byref(b)) == daq.DAQ_OK
        cap = 0 if N == 0 else (N - 1) // (pre + post + 2) + 1
        expect = (up(32) + up(4 * C) + up(24 * cap) + up(2 * C * ((N + 7) // 8 * 8))
                  + (up(2 * C * stride) if flags else 0))
        assert b.value == expect
    f = daq.daq_fill(0x1000, 10, 12, 1, 100, -200, 8, 24, 0)  # stride not a multiple of 8
    assert lib.daq_server_slot_bytes(ctypes.byref(f), 0, ctypes.byref(b)) == daq.DAQ_EALIGN
    f = daq.daq_fill(0x1000, 10, 16, 0, 100, -200, 8, 24, 0)  # no channels
    assert lib.daq_server_slot_bytes(ctypes.byref(f), 0, ctypes.byref(b)) == daq.DAQ_EINVAL
    f = daq.daq_fill(0x1000, 10, 16, 1, 100, -200, 8, 24, 0)
    assert lib.daq_server_slot_bytes(ctypes.byref(f), 4, ctypes.byref(b)) == daq.DAQ_EINVAL  # unknown flag
    assert lib.daq_server_slot_bytes(ctypes.byref(f), 3, ctypes.byref(b)) == daq.DAQ_EINVAL  # both host forms
    assert lib.daq_server_slot_bytes(ctypes.byref(f), 0, None) == daq.DAQ_EINVAL
    # 12-bit words: the raw rows and the packed rows
    f = daq.daq_fill(0x1000, 560_000, 560_000, 54, 100, -200, 8, 24, 0)
    assert lib.daq_server_slot_bytes(ctypes.byref(f), daq.DAQ_SUBMIT_HOST_PACKED12, ctypes.byref(b)) == daq.DAQ_OK
    cap = (560_000 - 1) // 34 + 1
    assert b.value == (up(32) + up(4 * 54) + up(24 * cap) + up(2 * 54 * 560_000) + up(2 * 54 * 560_000)
                       + up(54 * 840_000))


def test_packed12_stride():
    lib = daq.load_library()
    for n, want in ((0, 0), (1, 4), (2, 4), (3, 8), (8, 12), (9, 16), (560_000, 840_000)):
        assert lib.daq_packed12_stride(n) == want
    assert lib.daq_packed12_stride(-1) == -1


def test_server_calls_reject_null_handles_without_touching_a_gpu():
    lib = daq.load_library()
    h = ctypes.c_void_p()
    assert lib.daq_server_create(ctypes.byref(h), None, 0x1000, 1 << 20, 1, 1) == daq.DAQ_EINVAL
    assert lib.daq_server_create(None, None, 0x1000, 1 << 20, 1, 1) == daq.DAQ_EINVAL
    f = daq.daq_fill(0x1000, 10, 16, 1, 100, -200, 8, 24, 0)
    t = ctypes.c_uint64(0)
    assert lib.daq_submit_fill(None, ctypes.byref(f), 0, 0, ctypes.byref(t)) == daq.DAQ_EINVAL
    assert lib.daq_submit_fill_at(None, ctypes.byref(f), 0, 0, 0, ctypes.byref(t)) == daq.DAQ_EINVAL
    assert lib.daq_server_set_limits(None, 10, 10) == daq.DAQ_EINVAL
    assert lib.daq_read_stream(None, 1 << 20, None, 4, 0, None) == daq.DAQ_EINVAL
    assert lib.daq_read_tiles(None, 1, 54, 560_000, None, 4, 0, None, None) == daq.DAQ_EINVAL
    assert lib.daq_ctx_get_graphs(None, None) == daq.DAQ_EINVAL
    buf = (daq.daq_completion * 4)()
    assert lib.daq_poll(None, buf, 4, 0) == daq.DAQ_EINVAL
    assert lib.daq_release(None, 1) == daq.DAQ_EINVAL
    st = daq.daq_server_stats()
    assert lib.daq_server_get_stats(None, ctypes.byref(st)) == daq.DAQ_EINVAL
    lib.daq_server_destroy(None)
    d = ctypes.c_int(0)
    assert lib.daq_ctx_get_device(None, ctypes.byref(d)) == daq.DAQ_EINVAL


def test_server_struct_layouts():
    assert ctypes.sizeof(daq.daq_counts) == 24
    assert ctypes.sizeof(daq.daq_completion) == 8 + 8 + 24 + 48 + 8 + 4 + 4 + 24
    assert ctypes.sizeof(daq.daq_server_stats) == 8 * 8 + 8 + 4 * 8


def test_header_constants_match_the_binding():
    """Every #define DAQ_<NAME> <integer> of the header has the same value in the binding."""
    text = open(HEADER).read()
    found = re.findall(r"^#define (DAQ_[A-Z_0-9]+)\s+\(?(-?\d+)\)?", text, flags=re.M)
    assert len(found) > 15
    checked = 0
    for name, value in found:
        if hasattr(daq, name):
            assert getattr(daq, name) == int(value), name
            checked += 1
    for name in ("DAQ_VARIANT_SPLIT", "DAQ_VARIANT_PIPE", "DAQ_STATUS_CAPACITY", "DAQ_STATUS_OUT_STRIDE",
                 "DAQ_STATUS_INCOMPLETE", "DAQ_EINVAL"):
        assert hasattr(daq, name), name
    assert checked >= 10


def test_compress_descriptor_and_word_bound():
    """daq_z_fill is the 80-byte record the header states; the binding's word
    bound (34 per block) is what the widest block needs: 63 codes of 17 bits,
    which the oracle's encoder reaches on alternating int16 extremes."""
    import numpy as np
    import oracle
    assert ctypes.sizeof(daq.daq_z_fill) == 80
    x = np.where(np.arange(128) % 2, 32767, -32768).astype(np.int16)[None, :]
    hdr, words = oracle.z_compress(x)
    assert (hdr >> 16).tolist() == [daq.DAQ_Z_MAX_WIDTH] * 2
    assert len(words) == daq.z_words_bound(1, 128) == 68


def test_compress_rejects_bad_arguments_without_touching_a_gpu():
    lib = daq.load_library()
    assert lib.daq_compress_batch(None, None, 0, None) == daq.DAQ_EINVAL
    z = daq.daq_z_fill(0x1000, 8, 0x2000, 8, 0x3000, None, 0x4000, 16, 0x5000, 1, 0)
    assert lib.daq_compress_batch(None, (daq.daq_z_fill * 1)(z), 1, None) == daq.DAQ_EINVAL


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    """Without the built library the binding raises instead of falling back."""
    monkeypatch.setattr(daq, "LIB_PATH", str(tmp_path / "libdaqisland.so"))
    monkeypatch.setattr(daq, "_lib", None)
    with pytest.raises(ImportError):
        daq.load_library()
    with pytest.raises(ImportError):
        daq.Context(0)


def test_fused_call_rejects_bad_arguments_without_touching_a_gpu():
    lib = daq.load_library()
    f = (daq.daq_fill * 1)(daq.daq_fill(0x1000, 10, 16, 1, 100, -200, 8, 24, 0))
    o = (daq.daq_fill_out * 1)(daq.daq_fill_out(0x2000, 1, 0x3000, 0x4000, 0x5000, 16))
    q = (daq.daq_q_out * 1)(daq.daq_q_out(0x6000, 0x7000, 16, None))
    assert lib.daq_process_batch_q(None, f, o, q, 1, None) == daq.DAQ_EINVAL
    assert lib.daq_qmethod_batch(None, f, q, 1, None) == daq.DAQ_EINVAL


def _no_device_child(env_extra):
    """Runs daq_ctx_create in a child process (the library reads DAQ_LOG once
    per process) and returns (status, last HIP error, stderr)."""
    code = ("import ctypes, paper_1611_04959_amd as daq\n"
            "lib = ctypes.CDLL(daq.LIB_PATH)\n"
            "h = ctypes.c_void_p()\n"
            "print(lib.daq_ctx_create(ctypes.byref(h), 0), lib.daq_last_hip_error())\n")
    env = {k: v for k, v in os.environ.items() if k not in ("DAQ_LOG", "DAQ_SCHEDULE")}
    env.update(env_extra)
    env["PYTHONPATH"] = ROOT
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stderr[-2000:]
    rc, hip = (int(v) for v in r.stdout.split())
    return rc, hip, r.stderr


def test_failed_hip_call_is_logged_at_level_one():
    torch = pytest.importorskip("torch")
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present: daq_ctx_create succeeds")
    rc, hip, err = _no_device_child({"DAQ_LOG": "1"})
    assert rc == daq.DAQ_EHIP and hip != 0
    lines = [ln for ln in err.splitlines() if ln.startswith("[daq] ")]
    assert len(lines) == 1 and "hipGetDeviceCount" in lines[0] and "failed" in lines[0], err
    rc0, _, err0 = _no_device_child({})
    assert rc0 == daq.DAQ_EHIP
    assert "[daq]" not in err0
