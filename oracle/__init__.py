"""CPU oracle for T-method island chopping -- TEST INFRASTRUCTURE ONLY.

Plain, slow, single-threaded C (``chop_oracle.c``) wrapped with ctypes. It
states the paper's computation step by step (Table 2 rows and the T-method
paragraph of Section 3); see the header of ``chop_oracle.c`` for the steps
and the readings taken where the paper is silent.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. The HIP library shares no code with it.

Parity of every function here is pinned by ``tests/test_oracle_pins.py``
(brute force from the window definition, closed forms, hand-derived golden
fixtures, library sums and invariants).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "chop_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_i16p = ctypes.POINTER(ctypes.c_int16)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def build() -> str:
    """Compile ``liboracle.so`` with gcc (plain -O2, no vectorisation tricks)."""
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC",
                           "-shared", "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    _lib = _bind(_LIB)
    return _lib


def _bind(path):
    """Load a compiled copy of chop_oracle.c and declare its signatures."""
    lib = ctypes.CDLL(path)
    lib.orc_pedestals.argtypes = [_i16p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                  ctypes.c_int32, _i32p]
    lib.orc_pedestals.restype = None
    lib.orc_calo_sum.argtypes = [_i16p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                 _i32p, _i64p]
    lib.orc_calo_sum.restype = None
    lib.orc_threshold.argtypes = [_i64p, ctypes.c_int64, ctypes.c_int32, _u8p]
    lib.orc_threshold.restype = None
    lib.orc_dilate.argtypes = [_u8p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _u8p]
    lib.orc_dilate.restype = None
    lib.orc_islands.argtypes = [_u8p, ctypes.c_int64, _i64p, ctypes.c_int64, _i64p]
    lib.orc_islands.restype = ctypes.c_int64
    lib.orc_gather.argtypes = [_i16p, ctypes.c_int32, ctypes.c_int64, _i64p, ctypes.c_int64,
                               _i16p, ctypes.c_int64]
    lib.orc_gather.restype = None
    lib.orc_chop.argtypes = [_i16p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                             ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                             _i32p, _i64p, ctypes.c_int64, _i64p, _i16p, ctypes.c_int64]
    lib.orc_chop.restype = ctypes.c_int64
    lib.orc_q_decimate.argtypes = [_i64p, ctypes.c_int64, ctypes.c_int32, _i64p]
    lib.orc_q_decimate.restype = None
    lib.orc_q_accumulate.argtypes = [_i16p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, _i32p, _i32p,
                                     ctypes.c_int64]
    lib.orc_q_accumulate.restype = None
    lib.orc_qmethod.argtypes = [_i16p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                ctypes.c_int32, _i32p, _i64p, _i32p, ctypes.c_int64]
    lib.orc_qmethod.restype = ctypes.c_int
    lib.orc_unpack12.argtypes = [_u8p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, _i16p, ctypes.c_int64]
    lib.orc_unpack12.restype = None
    _u32p = ctypes.POINTER(ctypes.c_uint32)
    lib.orc_z_compress.argtypes = [_i16p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, _u32p, _u32p,
                                   ctypes.c_int64]
    lib.orc_z_compress.restype = ctypes.c_int64
    lib.orc_z_decompress.argtypes = [_u32p, _u32p, ctypes.c_int32, ctypes.c_int64, _i16p, ctypes.c_int64]
    lib.orc_z_decompress.restype = None
    return lib


def _ptr(a, typ):
    return a.ctypes.data_as(typ)


def _as_fill(x, n_samples):
    x = np.asarray(x)
    if x.dtype != np.int16 or x.ndim != 2:
        raise TypeError("fill must be a 2-D int16 array [channels, row_stride]")
    C, stride_avail = x.shape
    if stride_avail > 0 and x.strides[1] != 2:
        raise ValueError("fill rows must be contiguous")
    N = stride_avail if n_samples is None else int(n_samples)
    if N < 0 or N > stride_avail:
        raise ValueError("n_samples out of range")
    return x, C, N, (x.strides[0] // 2 if stride_avail > 0 else 0)


def pedestals(x, n_samples=None, ped_samples=100):
    """Table 2 pedestal row: int32[C], mean of the first ped_samples, rounded half up."""
    x, C, N, stride = _as_fill(x, n_samples)
    ped = np.zeros(C, np.int32)
    _load().orc_pedestals(_ptr(x, _i16p), C, N, stride, int(ped_samples), _ptr(ped, _i32p))
    return ped


def calo_sum(x, ped, n_samples=None):
    """Table 2 waveform-sum row: int64[N] pedestal-subtracted calorimeter sum."""
    x, C, N, stride = _as_fill(x, n_samples)
    ped = np.ascontiguousarray(ped, np.int32)
    S = np.zeros(max(N, 1), np.int64)
    _load().orc_calo_sum(_ptr(x, _i16p), C, N, stride, _ptr(ped, _i32p), _ptr(S, _i64p))
    return S[:N]


def threshold(S, thr):
    """Table 2 threshold row: uint8[N] flags S < thr."""
    S = np.ascontiguousarray(S, np.int64)
    F = np.zeros(max(len(S), 1), np.uint8)
    _load().orc_threshold(_ptr(S, _i64p), len(S), int(thr), _ptr(F, _u8p))
    return F[:len(S)]


def dilate(F, pre, post):
    """Table 2 pre/post-sample row: uint8[N] marks of the dilated windows."""
    F = np.ascontiguousarray(F, np.uint8)
    M = np.zeros(max(len(F), 1), np.uint8)
    _load().orc_dilate(_ptr(F, _u8p), len(F), int(pre), int(post), _ptr(M, _u8p))
    return M[:len(F)]


def islands(M, capacity=None):
    """Table 2 merge-check / island-array rows: (int64[n,3] records, total_len)."""
    M = np.ascontiguousarray(M, np.uint8)
    cap = len(M) // 2 + 1 if capacity is None else int(capacity)
    rec = np.zeros((max(cap, 1), 3), np.int64)
    total = np.zeros(1, np.int64)
    n = _load().orc_islands(_ptr(M, _u8p), len(M), _ptr(rec, _i64p), cap, _ptr(total, _i64p))
    return rec[:min(n, cap)].copy(), int(total[0]), int(n)


def gather(x, recs, out_stride=None):
    """Section 3 chopped islands: int16[C, out_stride] packed raw samples."""
    x, C, _, stride = _as_fill(x, None)
    recs = np.ascontiguousarray(recs, np.int64).reshape(-1, 3)
    total = int((recs[:, 1] - recs[:, 0]).sum()) if len(recs) else 0
    ost = total if out_stride is None else int(out_stride)
    out = np.zeros((C, max(ost, 1)), np.int16)
    _load().orc_gather(_ptr(x, _i16p), C, stride, _ptr(recs, _i64p), len(recs),
                       _ptr(out, _i16p), out.shape[1])
    return out[:, :ost]


class ChopResult:
    """Everything one fill yields: pedestals, island records, counts, packed samples."""

    __slots__ = ("ped", "islands", "n_islands", "total_len", "out")

    def __init__(self, ped, islands, n_islands, total_len, out):
        self.ped = ped
        self.islands = islands
        self.n_islands = n_islands
        self.total_len = total_len
        self.out = out


def chop(x, n_samples=None, ped_samples=100, threshold=-200, pre=8, post=24,
         capacity=None, gather=True):
    """All steps for one fill (C rows of int16, channel-major, any row stride)."""
    x, C, N, stride = _as_fill(x, n_samples)
    cap = (N // 2 + 1) if capacity is None else int(capacity)
    ped = np.zeros(C, np.int32)
    rec = np.zeros((max(cap, 1), 3), np.int64)
    total = np.zeros(1, np.int64)
    out = np.zeros((C, max(N, 1)), np.int16) if gather else None
    n = _load().orc_chop(_ptr(x, _i16p), C, N, stride, int(ped_samples), int(threshold),
                         int(pre), int(post), _ptr(ped, _i32p), _ptr(rec, _i64p), cap,
                         _ptr(total, _i64p),
                         _ptr(out, _i16p) if gather else ctypes.cast(None, _i16p),
                         out.shape[1] if gather else 0)
    if n < 0:
        raise MemoryError("oracle scratch allocation failed")
    tl = int(total[0])
    return ChopResult(ped, rec[:min(n, cap)].copy(), int(n), tl,
                      out[:, :tl].copy() if gather else None)


Q_DECIMATION = 32  # Table 2: 17.5k decimation threads for 560k samples


def q_decimate(S, D=Q_DECIMATION):
    """Table 2 decimation row: int64[ceil(N / D)] block sums of the calorimeter sum."""
    S = np.ascontiguousarray(S, np.int64)
    nb = (len(S) + D - 1) // D
    Q = np.zeros(max(nb, 1), np.int64)
    _load().orc_q_decimate(_ptr(S, _i64p), len(S), int(D), _ptr(Q, _i64p))
    return Q[:nb]


def q_accumulate(x, ped, acc, n_samples=None):
    """Table 2 fill-by-fill row: adds x[c][t] - ped[c] to acc[c][t] in place (int32, wraps)."""
    x, C, N, stride = _as_fill(x, n_samples)
    ped = np.ascontiguousarray(ped, np.int32)
    if acc.dtype != np.int32 or acc.ndim != 2 or acc.shape[0] != C or acc.shape[1] < N:
        raise ValueError("acc must be int32 [channels, >= n_samples]")
    if not acc.flags.c_contiguous:
        raise ValueError("acc must be contiguous")
    _load().orc_q_accumulate(_ptr(x, _i16p), C, N, stride, _ptr(ped, _i32p), _ptr(acc, _i32p), acc.shape[1])
    return acc


def qmethod(x, n_samples=None, ped_samples=100, acc=None, D=Q_DECIMATION):
    """Q-method for one fill: (ped, Q); acc (if given) is updated in place."""
    x, C, N, stride = _as_fill(x, n_samples)
    ped = np.zeros(C, np.int32)
    nb = (N + D - 1) // D
    Q = np.zeros(max(nb, 1), np.int64)
    if acc is not None and (acc.dtype != np.int32 or acc.ndim != 2 or acc.shape[0] != C
                            or acc.shape[1] < N or not acc.flags.c_contiguous):
        raise ValueError("acc must be contiguous int32 [channels, >= n_samples]")
    rc = _load().orc_qmethod(_ptr(x, _i16p), C, N, stride, int(ped_samples), int(D), _ptr(ped, _i32p),
                             _ptr(Q, _i64p), _ptr(acc, _i32p) if acc is not None else ctypes.cast(None, _i32p),
                             acc.shape[1] if acc is not None else 0)
    if rc != 0:
        raise MemoryError("oracle scratch allocation failed")
    return ped, Q[:nb].copy()


def packed12_row_bytes(n: int) -> int:
    """Bytes of one channel row of n samples in the 12-bit packing (two samples per three bytes)."""
    return (3 * int(n) + 1) // 2


def unpack12(packed, n_samples, out_stride=None):
    """Ingest: uint8 [C, row_bytes] 12-bit packed rows -> int16 [C, out_stride] (zero beyond n)."""
    packed = np.ascontiguousarray(packed, np.uint8)
    C, row_bytes = packed.shape
    if row_bytes < packed12_row_bytes(n_samples):
        raise ValueError("packed rows too short for n_samples")
    ost = int(n_samples) if out_stride is None else int(out_stride)
    out = np.zeros((C, max(ost, 1)), np.int16)
    _load().orc_unpack12(_ptr(packed, _u8p), row_bytes, C, int(n_samples), _ptr(out, _i16p), out.shape[1])
    return out[:, :ost]


Z_BLOCK = 64  # samples per compressed block


def z_compress(x, L=None):
    """Compression of C rows (int16 [C, >= L]): (hdr uint32 [C * ceil(L / 64)], words uint32 [n])."""
    x = np.ascontiguousarray(x, np.int16)
    C = x.shape[0]
    L = x.shape[1] if L is None else int(L)
    nb = (L + Z_BLOCK - 1) // Z_BLOCK
    hdr = np.zeros(max(C * nb, 1), np.uint32)
    cap = C * nb * 34 + 1                       # at most 17 bits per difference
    words = np.zeros(cap, np.uint32)
    u32 = ctypes.POINTER(ctypes.c_uint32)
    n = _load().orc_z_compress(_ptr(x, _i16p), C, L, x.shape[1], _ptr(hdr, u32), _ptr(words, u32), cap)
    return hdr[:C * nb].copy(), words[:n].copy()


def z_decompress(hdr, words, C, L):
    """Inverse of z_compress: int16 [C, L]."""
    hdr = np.ascontiguousarray(hdr, np.uint32)
    words = np.ascontiguousarray(words if len(words) else np.zeros(1, np.uint32), np.uint32)
    out = np.zeros((C, max(L, 1)), np.int16)
    u32 = ctypes.POINTER(ctypes.c_uint32)
    _load().orc_z_decompress(_ptr(hdr if len(hdr) else np.zeros(1, np.uint32), u32), _ptr(words, u32), C, int(L),
                             _ptr(out, _i16p), out.shape[1])
    return out[:, :L]
