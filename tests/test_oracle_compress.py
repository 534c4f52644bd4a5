"""Pins of the oracle's island compression (Section 3: the frontend's lossless
compression; delta + zigzag + per-block bit width, the reading documented in
the oracle), CPU only: a hand-worked block, an independent encoder written
here from the format (a Python big-integer bit stream), lossless round trips
over extremes and ragged lengths, the size formula, and planted mistakes."""
import os
import subprocess
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import oracle  # noqa: E402

SRC = os.path.join(os.path.dirname(oracle.__file__), "chop_oracle.c")
B = oracle.Z_BLOCK


def encode_ref(x, L):
    """Encoder from the format: per block first sample, w, then z_i at bits (i-1) w."""
    C = x.shape[0]
    nb = -(-L // B)
    hdr, words = [], []
    for c in range(C):
        for k in range(nb):
            v = [int(t) for t in x[c, k * B:min(L, k * B + B)]]
            z = []
            for i in range(1, len(v)):
                r = v[i] - v[i - 1]
                z.append(2 * r if r >= 0 else -2 * r - 1)
            w = max(z).bit_length() if z else 0
            hdr.append((v[0] & 0xFFFF) | (w << 16))
            stream = 0
            for i, zi in enumerate(z):
                stream |= zi << (i * w)
            for j in range(-(-len(z) * w // 32)):
                words.append((stream >> (32 * j)) & 0xFFFFFFFF)
    return hdr, words


def test_hand_worked_block():
    # [5, 7, 4]: differences 2, -3 -> zigzag 4, 5 -> 3 bits: 100, 101 -> 0b101100 = 44
    h, w = oracle.z_compress(np.array([[5, 7, 4]], np.int16))
    assert h.tolist() == [5 | 3 << 16] and w.tolist() == [44]
    assert oracle.z_decompress(h, w, 1, 3).tolist() == [[5, 7, 4]]
    # a constant block needs no payload; a one-sample block neither
    h, w = oracle.z_compress(np.full((2, 64), -9, np.int16))
    assert h.tolist() == [0xFFF7] * 2 and len(w) == 0
    h, w = oracle.z_compress(np.array([[123]], np.int16))
    assert h.tolist() == [123] and len(w) == 0


def test_matches_an_independent_encoder():
    rng = np.random.default_rng(8)
    for _ in range(200):
        C, L = int(rng.integers(1, 4)), int(rng.integers(0, 300))
        lo, hi = [(-5, 5), (-300, 300), (-32768, 32767)][int(rng.integers(0, 3))]
        x = rng.integers(lo, hi + 1, size=(C, max(L, 1))).astype(np.int16)
        h, w = oracle.z_compress(x, L)
        rh, rw = encode_ref(x, L)
        assert h.tolist() == rh and w.tolist() == rw


def test_lossless_round_trips():
    rng = np.random.default_rng(9)
    cases = [np.array([[-32768, 32767, -32768, 0, 32767]], np.int16),        # widest differences: 17 bits
             rng.integers(1700, 1900, size=(54, 6400)).astype(np.int16),
             rng.integers(-32768, 32768, size=(3, 1000)).astype(np.int16),
             np.zeros((2, 65), np.int16)]
    for x in cases:
        for L in (x.shape[1], x.shape[1] - 1, 1, 0):
            h, w = oracle.z_compress(x, L)
            assert (oracle.z_decompress(h, w, x.shape[0], L) == x[:, :L]).all()
    h, _ = oracle.z_compress(cases[0])
    assert (h[0] >> 16) == 17


def test_size_formula_and_ratio():
    spec = __import__("synth").config_c0()[0]
    x = __import__("synth").render(spec)
    r = oracle.chop(x, n_samples=spec.n_samples, ped_samples=spec.ped_samples, threshold=spec.threshold,
                    pre=spec.pre, post=spec.post)
    h, w = oracle.z_compress(r.out, r.total_len)
    L = r.total_len
    sizes = []
    for b, hb in enumerate(h.tolist()):
        n = min(B, L - (b % -(-L // B)) * B)
        sizes.append(-(-(n - 1) * (hb >> 16) // 32))
    assert len(w) == sum(sizes)
    compressed = 4 * (len(h) + len(w))
    assert 2 * r.out.size / compressed > 1.5      # island samples compress well
    assert (oracle.z_decompress(h, w, r.out.shape[0], L) == r.out).all()


def _pins_pass():
    try:
        test_hand_worked_block()
        test_matches_an_independent_encoder()
        test_lossless_round_trips()
    except AssertionError:
        return False
    return True


MUTANTS = {
    "zigzag_sign": ("uint32_t z = ((uint32_t)r << 1) ^ (uint32_t)(r >> 31);\n                if (z > zmax)",
                    "uint32_t z = ((uint32_t)r << 1);\n                if (z > zmax)"),
    "width_short": ("while (w < 32 && (zmax >> w) != 0)\n                w++;",
                    "while (w < 32 && (zmax >> w) > 1)\n                w++;"),
    "first_sample_dropped": ("hdr[(int64_t)c * nb + k] = (uint32_t)(uint16_t)row[t0] | (w << 16);",
                             "hdr[(int64_t)c * nb + k] = (w << 16);"),
    "bit_order": ("words[wi] |= 1u << (at % 32);", "words[wi] |= 1u << (31 - at % 32);"),
}


def test_unmutated_oracle_passes():
    assert _pins_pass()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site not found: %s" % name
    mpath = tmp_path / "mutant.c"
    mpath.write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-o", str(so), str(mpath)])
    saved = oracle._lib
    try:
        oracle._lib = oracle._bind(str(so))
        assert not _pins_pass(), "mutant %s survived the pins" % name
    finally:
        oracle._lib = saved
