"""The pins catch plausible mistakes in the oracle.

Each case plants one mistake in a copy of the oracle's C source (on the CPU,
in a temporary directory), builds it, points the oracle module at it and
runs a fast subset of the pins; at least one pin must fail. Mutations that
would write out of bounds are not planted.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import oracle  # noqa: E402
import test_oracle_pins as pins  # noqa: E402
import golden_io  # noqa: E402

SRC = os.path.join(os.path.dirname(oracle.__file__), "chop_oracle.c")

MUTANTS = {
    "non_strict_threshold": ("(S[t] < (int64_t)thr)", "(S[t] <= (int64_t)thr)"),
    "pre_post_swapped": ("int64_t lo = t - pre;\n        int64_t hi = t + post;",
                         "int64_t lo = t - post;\n        int64_t hi = t + pre;"),
    "truncated_mean": ("floor_div(2 * P + n, 2 * n)", "floor_div(P, n)"),
    "round_toward_zero": ("if ((a % b) != 0 && (a < 0))", "if (0)"),
    "pedestal_not_subtracted": ("S[t] = s - ped_total;", "S[t] = s;"),
    "channel_dropped": ("        for (int32_t c = 0; c < C; c++)\n            s += x",
                        "        for (int32_t c = 1; c < C; c++)\n            s += x"),
    "inclusive_stop": ("islands[3 * n + 1] = t;", "islands[3 * n + 1] = t - 1;"),
    "offset_off_by_one": ("offset += t - start;", "offset += t - start + (n > 0);"),
    "window_short_by_one": ("for (int64_t u = lo; u <= hi; u++)", "for (int64_t u = lo; u < hi; u++)"),
    "gather_wrong_index": ("x[(int64_t)c * stride + start + k];", "x[(int64_t)c * stride + start];"),
    "ped_over_Np_not_n": ("ped[c] = (int32_t)floor_div(2 * P + n, 2 * n);",
                          "ped[c] = (int32_t)floor_div(2 * P + Np, 2 * (int64_t)Np);"),
}


def _pins_pass():
    """Fast subset of the pins; True when all hold."""
    try:
        for path in golden_io.fixture_files():
            pins.test_golden_fixture(path)
        rng = np.random.default_rng(77)
        import brute
        for _ in range(600):
            x, N, Np, thr, pre, post = pins._random_case(rng)
            r = oracle.chop(x, n_samples=N, ped_samples=Np, threshold=thr, pre=pre, post=post)
            ped, isl, total, out, *_ = brute.chop(x.tolist(), N, Np, thr, pre, post)
            assert r.ped.tolist() == ped
            assert r.islands.tolist() == [list(i) for i in isl]
            assert r.total_len == total and r.out.tolist() == out
        pins.test_pedestal_short_fill_and_empty()
        pins.test_equal_to_threshold_is_not_a_crossing()
    except AssertionError:
        return False
    return True


def test_unmutated_oracle_passes_subset():
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
