"""Seeded synthetic calorimeter fills shaped like the paper's workload.

The paper's own inputs (its data simulator and SLAC test-beam data, Section 3)
are not available; these fills stand in for them. ``fillgen.c`` renders the
samples; this module holds the workload recipes (fill shapes, pulse rates and
chopping parameters of each benchmark configuration) and builds the C code.

It holds none of the island-chopping arithmetic. Tests, the benchmark and the
smoke check feed the same buffers to the HIP library and to the CPU oracle.
"""
from __future__ import annotations

import ctypes
import dataclasses
import hashlib
import os
import subprocess
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fillgen.c")
_LIB = os.path.join(_HERE, "libfillgen.so")
_lib = None

#: channels per calorimeter: a 6 x 9 grid of crystals (Section 3)
GRID_ROWS, GRID_COLS = 6, 9
CHANNELS = GRID_ROWS * GRID_COLS
#: samples per fill: 700 us at 800 MSPS (Section 3, Table 2 thread counts)
FILL_SAMPLES = 560_000
#: muon lifetime in the lab, 64.4 us, in 1.25 ns samples
TAU_SAMPLES = 51_520.0
#: initial pulse rate per sample giving about 2000 pulses per 560k-sample fill
LAMBDA0 = 0.03882


class _Params(ctypes.Structure):
    _fields_ = [("grid_rows", ctypes.c_int32), ("grid_cols", ctypes.c_int32),
                ("n_samples", ctypes.c_int64), ("row_stride", ctypes.c_int64),
                ("rate_mult", ctypes.c_double), ("lambda0", ctypes.c_double),
                ("tau_samples", ctypes.c_double), ("amp_lo", ctypes.c_double),
                ("amp_hi", ctypes.c_double), ("ped_lo", ctypes.c_double),
                ("ped_hi", ctypes.c_double), ("noise_sigma", ctypes.c_double),
                ("rise_sigma", ctypes.c_double), ("fall_tau", ctypes.c_double),
                ("max_crystals", ctypes.c_int32), ("adc_max", ctypes.c_int32)]


PULSE_DTYPE = np.dtype([("t0", "<f8"), ("amp", "<f8"), ("n_cry", "<i4"), ("cry", "<i4", (4,)),
                        ("frac", "<f8", (4,))], align=True)


def build() -> str:
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-ffp-contract=off", "-Wall", "-fPIC",
                           "-shared", "-pthread", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.synth_fill.argtypes = [ctypes.c_uint64, ctypes.POINTER(_Params),
                                   ctypes.POINTER(ctypes.c_int16), ctypes.c_void_p,
                                   ctypes.c_int64, ctypes.c_int32]
        lib.synth_fill.restype = ctypes.c_int64
        _lib = lib
    return _lib


def padded(n: int, multiple: int = 8) -> int:
    """Row stride: n rounded up to a whole number of 16-byte vectors."""
    return (int(n) + multiple - 1) // multiple * multiple


def fill_seed(config: str, stream: int, index: int) -> int:
    """64-bit fill seed from (configuration name, stream, fill index)."""
    h = hashlib.blake2b(f"{config}/{stream}/{index}".encode(), digest_size=8).digest()
    return int.from_bytes(h, "little")


@dataclasses.dataclass
class FillSpec:
    """One calorimeter fill: how to render it and how to chop it."""
    seed: int
    n_samples: int = FILL_SAMPLES
    rate: float = 1.0
    threshold: int = -200
    pre: int = 8
    post: int = 24
    ped_samples: int = 100
    n_channels: int = CHANNELS

    @property
    def row_stride(self) -> int:
        return padded(self.n_samples)

    @property
    def raw_bytes(self) -> int:
        return 2 * self.n_channels * self.n_samples


def render(spec: FillSpec, out: Optional[np.ndarray] = None, nthreads: Optional[int] = None,
           truth: bool = False, noise_sigma: float = 3.0):
    """Render one fill into ``out`` (int16 [54, row_stride], C-contiguous rows).

    Returns the array (and the truth pulse list when ``truth``)."""
    if spec.n_channels != CHANNELS:
        raise ValueError("the synthetic calorimeter has %d channels" % CHANNELS)
    stride = spec.row_stride
    if out is None:
        out = np.empty((CHANNELS, stride), np.int16)
    if out.dtype != np.int16 or out.shape != (CHANNELS, stride) or not out.flags.c_contiguous:
        raise ValueError("out must be C-contiguous int16 [%d, %d]" % (CHANNELS, stride))
    p = _Params(GRID_ROWS, GRID_COLS, spec.n_samples, stride, float(spec.rate), LAMBDA0,
                TAU_SAMPLES, 50.0, 3000.0, 1700.0, 1900.0, float(noise_sigma), 2.0, 6.0, 4, 4095)
    nt = nthreads or min(16, os.cpu_count() or 1)
    cap = 0
    tr = None
    if truth:
        cap = int(spec.rate * LAMBDA0 * TAU_SAMPLES * 1.5) + 200
        tr = np.zeros(cap, PULSE_DTYPE)
    n = _load().synth_fill(spec.seed, ctypes.byref(p),
                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_int16)),
                           tr.ctypes.data if truth else None, cap, nt)
    if n < 0:
        raise RuntimeError("synth_fill failed (%d)" % n)
    if truth:
        if n > cap:
            raise RuntimeError("truth list overflow")
        return out, tr[:n].copy()
    return out


# ---------------------------------------------------------------------------
# Workload recipes. c0..c4 follow the five benchmark configurations of the
# build: shapes from Section 3 (54 channels, 560,000 samples, 12-bit ADC).
# ---------------------------------------------------------------------------

def config_c0(index: int = 0) -> List[FillSpec]:
    """Plain: one 54 x 560,000 fill, 1x rate, thr -200, pre 8, post 24."""
    return [FillSpec(seed=fill_seed("c0", 0, index))]


def config_c1(n_fills: int = 16) -> List[FillSpec]:
    """16 fills of the c0 shape at 3x the initial pulse rate (frequent pileup)."""
    return [FillSpec(seed=fill_seed("c1", 0, i), rate=3.0) for i in range(n_fills)]


def config_c2(n_streams: int = 24, seed: int = 2) -> List[FillSpec]:
    """Uneven batch: per stream N ~ U{100k..560k}, rate ~ U(0.5, 4),
    thr ~ U{-400..-150}, pre ~ U{4..16}, post ~ U{16..48}."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_streams):
        out.append(FillSpec(seed=fill_seed("c2", s, 0),
                            n_samples=int(rng.integers(100_000, 560_001)),
                            rate=float(rng.uniform(0.5, 4.0)),
                            threshold=int(rng.integers(-400, -149)),
                            pre=int(rng.integers(4, 17)),
                            post=int(rng.integers(16, 49))))
    return out


def config_c3_fill(stream: int, index: int) -> FillSpec:
    """Serving: c0-distributed fills from 24 streams."""
    return FillSpec(seed=fill_seed("c3", stream, index))


def config_c4(n_fills: int = 4, n_calos: int = 24) -> List[FillSpec]:
    """Stress: the whole detector (24 calorimeters x 54 channels) per fill,
    10x rate, thr -100, post 48; every calorimeter is its own 54-channel unit."""
    return [FillSpec(seed=fill_seed("c4", cal, f), rate=10.0, threshold=-100, pre=8, post=48)
            for f in range(n_fills) for cal in range(n_calos)]


# ---------------------------------------------------------------------------
# Staging: host arrays for a list of fills, and their device copies.
# ---------------------------------------------------------------------------

def render_many(specs: List[FillSpec], nthreads: Optional[int] = None) -> List[np.ndarray]:
    """One host array [54, row_stride] per spec."""
    return [render(s, nthreads=nthreads) for s in specs]


def to_device(arrays: List[np.ndarray], device="cuda"):
    """Device copies (torch.int16, same shape); synchronises the copies."""
    import torch
    out = [torch.from_numpy(a).to(device) for a in arrays]
    torch.cuda.synchronize()
    return out
