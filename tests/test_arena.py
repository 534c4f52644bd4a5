"""The serving loop's arena bookkeeping (host C++, daqk::Arena), on the CPU.

Random allocate/release sequences are checked against brute force over the
set of live blocks: blocks are aligned, inside the budget and disjoint, each
allocation is the lowest offset with a large enough gap (first fit), and a
fully released arena is one free range again."""
import os
import random
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ALIGN = 256


@pytest.fixture(scope="module")
def arena_bin(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("arena") / "arena_check")
    subprocess.run(["g++", "-O1", "-std=c++17", "-fsanitize=address,undefined",
                    "-I", os.path.join(ROOT, "paper_1611_04959_amd", "csrc"),
                    os.path.join(ROOT, "tests", "native", "arena_check.cpp"), "-o", exe], check=True)
    return exe


def run(exe, size, ops):
    text = "\n".join(ops) + "\n"
    out = subprocess.run([exe, str(size)], input=text, capture_output=True, text=True, check=True).stdout
    return out.split("\n")


def first_fit(live, size, n):
    """Lowest aligned offset where n bytes fit between the live blocks."""
    pos = 0
    for off, length in sorted(live.items()):
        if off - pos >= n:
            return pos
        pos = max(pos, off + length)
    return pos if size - pos >= n else -1


@pytest.mark.parametrize("seed", range(6))
def test_random_sequences_match_first_fit(arena_bin, seed):
    rng = random.Random(seed)
    size = rng.choice([1 << 16, 1 << 20, 10_000_000]) // ALIGN * ALIGN
    live, ops, expect = {}, [], []
    # build the op list with the model, then replay it through the binary
    for _ in range(600):
        if live and rng.random() < 0.45:
            off = rng.choice(sorted(live))
            ops.append("r %d" % off)
            expect.append(("r", off, 1))
            del live[off]
        else:
            n = rng.choice([1, 255, 256, 257, rng.randrange(1, size // 8 + 2), rng.randrange(1, 5000)])
            rn = (n + ALIGN - 1) // ALIGN * ALIGN
            got = first_fit(live, size, rn)
            ops.append("a %d" % n)
            expect.append(("a", n, got))
            if got >= 0:
                live[got] = rn
    ops.append("s")
    lines = run(arena_bin, size, ops)
    for (kind, arg, want), line in zip(expect, lines):
        assert int(line) == want, (kind, arg)
    in_use, peak, largest, ranges, blocks = (int(v) for v in lines[len(expect)].split())
    assert in_use == sum(live.values())
    assert blocks == len(live)
    assert peak >= in_use


def test_blocks_are_aligned_disjoint_and_inside(arena_bin):
    size = 1 << 20
    ops = ["a %d" % n for n in (1, 300, 256, 5000, 77, 100000, 1)]
    offs = [int(v) for v in run(arena_bin, size, ops)[:len(ops)]]
    spans = []
    for n, off in zip((1, 300, 256, 5000, 77, 100000, 1), offs):
        assert off >= 0 and off % ALIGN == 0
        end = off + (n + ALIGN - 1) // ALIGN * ALIGN
        assert end <= size
        spans.append((off, end))
    spans.sort()
    for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
        assert a1 <= b0


def test_release_merges_neighbours_back_to_one_range(arena_bin):
    size = 64 * ALIGN
    ops = ["a %d" % ALIGN for _ in range(64)] + ["a 1"]
    # release in an order that exercises merging on both sides
    order = list(range(0, 64, 2)) + list(range(1, 64, 2))
    ops += ["r %d" % (i * ALIGN) for i in order] + ["s", "a %d" % size, "r 0", "r 0", "r 12345", "s"]
    lines = run(arena_bin, size, ops)
    assert [int(v) for v in lines[:64]] == [i * ALIGN for i in range(64)]
    assert int(lines[64]) == -1  # full
    assert all(int(v) == 1 for v in lines[65:129])
    in_use, peak, largest, ranges, blocks = (int(v) for v in lines[129].split())
    assert (in_use, peak, largest, ranges, blocks) == (0, size, size, 1, 0)
    assert int(lines[130]) == 0          # the whole budget in one block
    assert int(lines[131]) == 1 and int(lines[132]) == 0 and int(lines[133]) == 0
    assert lines[134].split()[:4] == ["0", str(size), str(size), "1"]


def test_zero_and_oversized_requests(arena_bin):
    lines = run(arena_bin, 4096, ["a 0", "a 4097", "a 4096", "a 1"])
    assert [int(v) for v in lines[:4]] == [-1, -1, 0, -1]
