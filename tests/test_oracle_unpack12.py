"""Pins of the oracle's 12-bit ingest unpacking (Section 3: 12-bit
digitizers; two samples per three bytes, little-endian), CPU only: a
hand-worked byte example, a round trip through a packer written here from
the layout (bit by bit, not by the oracle's formula), odd lengths, the value
range, and planted mistakes."""
import os
import subprocess
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import oracle  # noqa: E402

SRC = os.path.join(os.path.dirname(oracle.__file__), "chop_oracle.c")


def pack_bits(x):
    """Reference packer: the row's samples as a little-endian bit stream, 12 bits each."""
    C, n = x.shape
    nbytes = oracle.packed12_row_bytes(n)
    out = np.zeros((C, max(nbytes, 1)), np.uint8)
    for c in range(C):
        bits = 0
        for t in range(n):
            bits |= (int(x[c, t]) & 0xFFF) << (12 * t)
        for b in range(nbytes):
            out[c, b] = (bits >> (8 * b)) & 0xFF
    return out


def test_hand_worked_bytes():
    # 0xABC, 0x123 -> BC, (A | 3 << 4) = 3A, 12
    assert oracle.unpack12(np.array([[0xBC, 0x3A, 0x12]], np.uint8), 2).tolist() == [[0xABC, 0x123]]
    # an odd last sample uses the low nibble of its second byte only
    assert oracle.unpack12(np.array([[0xFF, 0x0F]], np.uint8), 1).tolist() == [[4095]]
    assert oracle.packed12_row_bytes(1) == 2 and oracle.packed12_row_bytes(2) == 3
    assert oracle.packed12_row_bytes(7) == 11 and oracle.packed12_row_bytes(560_000) == 840_000


def test_round_trip_against_a_bit_stream_packer():
    rng = np.random.default_rng(2)
    for n in (0, 1, 2, 3, 7, 8, 15, 16, 17, 101):
        x = rng.integers(0, 4096, size=(3, max(n, 1))).astype(np.int16)[:, :max(n, 1)]
        p = pack_bits(x[:, :n])
        got = oracle.unpack12(p, n) if n else np.zeros((3, 0), np.int16)
        assert got.tolist() == x[:, :n].tolist()


def test_extremes_and_row_strides():
    x = np.array([[0, 4095, 1, 4094, 2048, 2047, 0, 4095, 7]], np.int16)
    p = pack_bits(x)
    wide = np.zeros((1, p.shape[1] + 5), np.uint8)
    wide[:, :p.shape[1]] = p
    assert oracle.unpack12(wide, 9).tolist() == x.tolist()
    out = oracle.unpack12(wide, 9, out_stride=16)
    assert out[:, :9].tolist() == x.tolist() and not out[:, 9:].any()


def _pins_pass():
    try:
        test_hand_worked_bytes()
        test_round_trip_against_a_bit_stream_packer()
        test_extremes_and_row_strides()
    except AssertionError:
        return False
    return True


MUTANTS = {
    "nibbles_swapped": ("out[t] = (int16_t)(p[0] | ((p[1] & 0x0F) << 8));",
                        "out[t] = (int16_t)(p[0] | ((p[1] >> 4) << 8));"),
    "byte_order": ("out[t] = (int16_t)((p[1] >> 4) | (p[2] << 4));",
                   "out[t] = (int16_t)((p[2] >> 4) | (p[1] << 4));"),
    "pair_stride": ("const uint8_t *p = in + 3 * k;", "const uint8_t *p = in + 2 * k;"),
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
