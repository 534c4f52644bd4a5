"""The boundary from plain C: tests/native/c_client.c (built by
__graft_entry__.build()) includes only include/daq.h and HIP's C runtime API,
chops one synthetic fill with daq_chop_fill and compresses the packed rows
with daq_compress_batch. Its output must equal the oracle's chop and
compression, element by element."""
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLIENT = os.path.join(ROOT, "tests", "native", "c_client")


def read_output(path, C):
    b = open(path, "rb").read()
    at = 0

    def take(dtype, count):
        nonlocal at
        a = np.frombuffer(b, dtype, count, at)
        at += a.nbytes
        return a

    n, total, status = take("<i8", 3).tolist()
    ped = take("<i4", C)
    isl = take("<i8", 3 * n).reshape(n, 3)
    packed = take("<i2", C * total).reshape(C, total)
    n_words = int(take("<i8", 1)[0])
    nb = C * ((total + oracle.Z_BLOCK - 1) // oracle.Z_BLOCK)
    hdr = take("<u4", nb)
    words = take("<u4", n_words)
    assert at == len(b)
    return n, total, status, ped, isl, packed, hdr, words


@pytest.mark.parametrize("n_samples,rate,thr", [(200_003, 3.0, -200), (4_001, 1.0, -150)])
def test_c_client_matches_oracle(tmp_path, n_samples, rate, thr):
    if not os.path.exists(CLIENT):
        pytest.skip("tests/native/c_client is not built (run __graft_entry__.build())")
    spec = synth.FillSpec(seed=synth.fill_seed("c-client", 0, n_samples), n_samples=n_samples, rate=rate,
                          threshold=thr)
    x = synth.render(spec)
    C = x.shape[0]
    src, dst = tmp_path / "fill.bin", tmp_path / "out.bin"
    x.tofile(src)
    args = [CLIENT, str(src), str(dst), str(C), str(n_samples), str(thr), str(spec.pre), str(spec.post),
            str(spec.ped_samples)]
    print("[gpu-test] c_client N=%d rate=%.1f thr=%d" % (n_samples, rate, thr), flush=True)
    r = subprocess.run(args, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    n, total, status, ped, isl, packed, hdr, words = read_output(dst, C)
    ref = oracle.chop(x, n_samples=n_samples, ped_samples=spec.ped_samples, threshold=thr, pre=spec.pre,
                      post=spec.post)
    assert status == 0
    assert (n, total) == (ref.n_islands, ref.total_len)
    np.testing.assert_array_equal(ped, ref.ped)
    np.testing.assert_array_equal(isl, ref.islands)
    np.testing.assert_array_equal(packed, ref.out)
    hdr_ref, words_ref = oracle.z_compress(ref.out, ref.total_len)
    np.testing.assert_array_equal(hdr, hdr_ref)
    np.testing.assert_array_equal(words, words_ref)
    assert n > 10
