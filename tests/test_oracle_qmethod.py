"""Pins of the oracle's Q-method (Table 2, decimation and fill-by-fill rows;
Section 3, Q-method paragraph), CPU only.

The decimated sum and the accumulator are pinned against closed forms (a
ramp whose pedestal, block sums and accumulator follow by hand), library
sums, the relation between the two outputs, brute force on tiny inputs,
order independence of accumulation and the int32 wrap. A last set of cases
plants mistakes in a copy of the oracle and checks that a pin fails.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import oracle  # noqa: E402

D = oracle.Q_DECIMATION
SRC = os.path.join(os.path.dirname(oracle.__file__), "chop_oracle.c")


def test_decimation_factor_is_the_papers():
    # Table 2: 17.5k decimation threads for 560k samples per fill
    assert D == 560_000 // 17_500 == 32


def test_ramp_closed_form():
    """x[c][t] = a_c + t, Np = 4: ped = a_c + 2 (mean a_c + 1.5 rounded half up),
    S[t] = C (t - 2), Q[b] = C (1024 b + 432) for whole blocks, and the
    six-sample tail t = 64..69 of N = 70 gives C (399 - 12)."""
    C, N = 3, 70
    a = np.array([100, -7, 2000])
    x = (a[:, None] + np.arange(N)[None, :]).astype(np.int16)
    acc = np.zeros((C, N), np.int32)
    ped, Q = oracle.qmethod(x, N, ped_samples=4, acc=acc)
    assert ped.tolist() == (a + 2).tolist()
    assert Q.tolist() == [C * 432, C * (1024 + 432), C * 387]
    assert acc.tolist() == [list(range(-2, N - 2))] * C


def test_constant_channels_give_zero():
    x = np.tile(np.array([[5], [1800], [-3]], np.int16), (1, 1000))
    acc = np.full((3, 1000), 17, np.int32)
    ped, Q = oracle.qmethod(x, 1000, acc=acc)
    assert ped.tolist() == [5, 1800, -3]
    assert not Q.any() and (acc == 17).all()


def _random(rng, C, N, lo=1700, hi=1900):
    return rng.integers(lo, hi, size=(C, N)).astype(np.int16)


def test_sums_and_the_two_outputs_agree():
    rng = np.random.default_rng(3)
    for C, N in ((1, 1), (2, 31), (5, 32), (7, 33), (54, 4097), (3, 100_001)):
        x = _random(rng, C, N)
        acc = np.zeros((C, N), np.int32)
        ped, Q = oracle.qmethod(x, N, ped_samples=int(rng.integers(1, 150)), acc=acc)
        assert len(Q) == -(-N // D)
        # library sums: the blocks add up to the whole calorimeter sum
        assert int(Q.sum()) == int(x.astype(np.int64).sum()) - N * int(ped.astype(np.int64).sum())
        # the accumulator's channel sum over each block is that block of Q
        col = acc.astype(np.int64).sum(0)
        pad = np.zeros(len(Q) * D, np.int64)
        pad[:N] = col
        assert pad.reshape(-1, D).sum(1).tolist() == Q.tolist()


def test_brute_force_tiny():
    rng = np.random.default_rng(11)
    for _ in range(300):
        C, N = int(rng.integers(1, 5)), int(rng.integers(0, 80))
        Np = int(rng.integers(1, 20))
        x = rng.integers(-50, 50, size=(C, max(N, 1))).astype(np.int16)
        xs = x.tolist()
        n = min(Np, N)
        ped = []
        for c in range(C):
            if n == 0:
                ped.append(0)
                continue
            P = sum(xs[c][:n])
            ped.append((2 * P + n) // (2 * n))   # Python // is the mathematical floor
        S = [sum(xs[c][t] for c in range(C)) - sum(ped) for t in range(N)]
        Qb = [sum(S[t] for t in range(b * D, min(b * D + D, N))) for b in range(-(-N // D))]
        acc0 = rng.integers(-1000, 1000, size=(C, max(N, 1))).astype(np.int32)
        acc = acc0.copy()
        p2, Q = oracle.qmethod(x, N, ped_samples=Np, acc=acc)
        assert p2.tolist() == ped and Q.tolist() == Qb
        want = [[acc0[c][t] + xs[c][t] - ped[c] if t < N else acc0[c][t] for t in range(acc0.shape[1])]
                for c in range(C)]
        assert acc.tolist() == want
        for d in (1, 2, 3, 7):
            assert oracle.q_decimate(np.array(S, np.int64), d).tolist() == \
                [sum(S[b * d:b * d + d]) for b in range(-(-N // d))]


def test_accumulation_is_order_free_and_linear():
    rng = np.random.default_rng(5)
    xa, xb = _random(rng, 4, 777), _random(rng, 4, 777)
    a1 = np.zeros((4, 777), np.int32)
    a2 = np.zeros((4, 777), np.int32)
    oracle.qmethod(xa, acc=a1)
    oracle.qmethod(xb, acc=a1)
    oracle.qmethod(xb, acc=a2)
    oracle.qmethod(xa, acc=a2)
    assert (a1 == a2).all()
    a3 = np.zeros((4, 777), np.int32)
    for _ in range(5):
        ped, _ = oracle.qmethod(xa, acc=a3)
    assert (a3 == 5 * (xa.astype(np.int32) - ped[:, None])).all()


def test_accumulator_wraps_modulo_2_32():
    x = np.array([[0, 0, 1, -1]], np.int16)
    acc = np.array([[0, 0, 2**31 - 1, -2**31]], np.int32)
    oracle.qmethod(x, 4, ped_samples=2, acc=acc)   # ped = 0
    assert acc.tolist() == [[0, 0, -2**31, 2**31 - 1]]


def test_empty_and_short_fills():
    x = np.zeros((2, 8), np.int16)
    acc = np.full((2, 8), 9, np.int32)
    ped, Q = oracle.qmethod(x, 0, acc=acc)
    assert ped.tolist() == [0, 0] and len(Q) == 0 and (acc == 9).all()
    x = np.array([[3, 4, 5]], np.int16)
    ped, Q = oracle.qmethod(x, 3, ped_samples=100)   # N < Np: mean of the 3 samples
    assert ped.tolist() == [4] and Q.tolist() == [0]


def _pins_pass():
    try:
        test_ramp_closed_form()
        test_constant_channels_give_zero()
        test_sums_and_the_two_outputs_agree()
        test_accumulation_is_order_free_and_linear()
        test_accumulator_wraps_modulo_2_32()
        test_empty_and_short_fills()
    except AssertionError:
        return False
    return True


MUTANTS = {
    "blocks_shifted": ("Q[t / D] += S[t];", "Q[(t + 1) / D < nb ? (t + 1) / D : nb - 1] += S[t];"),
    "tail_block_dropped": ("    for (int64_t t = 0; t < N; t++)\n        Q[t / D] += S[t];",
                           "    for (int64_t t = 0; t < N / D * D; t++)\n        Q[t / D] += S[t];"),
    "acc_without_pedestal": ("int64_t v = (int64_t)x[(int64_t)c * stride + t] - ped[c];",
                             "int64_t v = (int64_t)x[(int64_t)c * stride + t];"),
    "acc_overwrites": ("acc[(int64_t)c * acc_stride + t] = (int32_t)(a + (uint32_t)v);",
                       "acc[(int64_t)c * acc_stride + t] = (int32_t)(0 * a + (uint32_t)v);"),
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
