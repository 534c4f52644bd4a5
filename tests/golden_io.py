"""Reader for the hand-derived fixtures in tests/golden/."""
import glob
import os

import numpy as np

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(path):
    d = {"x": [], "out": []}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, _, val = line.partition(":")
            key, val = key.strip(), val.strip()
            if key in ("x", "out"):
                d[key].append([int(v) for v in val.split()])
            elif key == "islands":
                recs = [tuple(int(v) for v in part.split()) for part in val.split(";") if part.strip()]
                d[key] = np.array(recs, np.int64).reshape(-1, 3)
            elif key == "ped":
                d[key] = np.array([int(v) for v in val.split()], np.int32)
            elif key in ("name", "cite"):
                d[key] = val
            else:
                d[key] = int(val)
    d["x"] = np.array(d["x"], np.int16)
    C = d["channels"]
    assert d["x"].shape == (C, d["samples"]), path
    d["out"] = (np.array(d["out"], np.int16) if d["out"]
                else np.zeros((C, 0), np.int16))
    return d


def all_fixtures():
    return sorted(glob.glob(os.path.join(GOLDEN_DIR, "*.txt")))


def fixture_files():
    return [p for p in all_fixtures() if not p.endswith("README.txt")]
