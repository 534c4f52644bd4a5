"""Brute-force statement of island chopping for tiny fills (pure Python).

Independent of the oracle's C code and written from a different formulation:
a sample is inside an island when some flagged sample lies in the window
[t - post, t + pre] around it (the set of samples that could have marked t),
pedestals use exact rational rounding, and islands are read off with
itertools.groupby. Only for fills of a few hundred samples.
"""
from fractions import Fraction
from itertools import groupby
import math


def pedestal(row, ped_samples):
    n = min(ped_samples, len(row))
    if n == 0:
        return 0
    mean = Fraction(sum(int(v) for v in row[:n]), n)
    return math.floor(mean + Fraction(1, 2))


def chop(x, n_samples, ped_samples, threshold, pre, post):
    """x: list of channel rows (ints). Returns (ped, islands, total_len, out)."""
    N = n_samples
    ped = [pedestal(list(r)[:N], ped_samples) for r in x]
    PED = sum(ped)
    S = [sum(int(r[t]) for r in x) - PED for t in range(N)]
    F = [s < threshold for s in S]
    M = [any(F[u] for u in range(t - post, t + pre + 1) if 0 <= u < N) for t in range(N)]
    islands = []
    t = 0
    offset = 0
    for key, grp in groupby(range(N), key=lambda i: M[i]):
        idx = list(grp)
        if key:
            islands.append((idx[0], idx[-1] + 1, offset))
            offset += len(idx)
    out = [[int(r[t]) for (s, e, _) in islands for t in range(s, e)] for r in x]
    return ped, islands, offset, out, S, F, M
