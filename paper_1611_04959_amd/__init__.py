"""Python binding of libdaqisland (include/daq.h): T-method island chopping of
waveform-digitizer fills on MI355X (gfx950).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libdaqisland.so``. PyTorch supplies device memory and streams.
The functions keep the C names; ``Context`` wraps a ``daq_ctx``.

Layouts (device tensors, ``torch.int16`` etc. on a ROCm device):
  raw      int16 [C, row_stride]  channel-major fill, row_stride % 8 == 0
  islands  int64 [capacity, 3]    (start, stop, offset) per island
  counts   int64 [3]              n_islands, total_len, status (low 32 bits)
  ped      int32 [C]              pedestals (optional)
  out      int16 [C, out_stride]  packed island samples (optional)
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import List, Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdaqisland.so")

DAQ_OK = 0
DAQ_EINVAL = -1
DAQ_EALIGN = -2
DAQ_EHIP = -3
DAQ_ENOMEM = -4
DAQ_EAGAIN = -5
DAQ_ERANGE = -6
DAQ_EMISMATCH = -7
DAQ_ETIMEDOUT = -8
DAQ_STATUS_CAPACITY = 1
DAQ_STATUS_OUT_STRIDE = 2
DAQ_STATUS_INCOMPLETE = 4
DAQ_MAX_WINDOW = 32768
DAQ_MAX_SAMPLES = 0x7FFFFFFF
DAQ_MAX_CHANNELS = 65535
DAQ_VARIANT_RELOAD = 0
DAQ_VARIANT_REGISTERS = 1
DAQ_VARIANT_LDS = 2
DAQ_VARIANT_RELOAD18 = 3
DAQ_VARIANT_RELOAD27 = 4
DAQ_VARIANT_SPLIT = 5
DAQ_VARIANT_PIPE = 6


class daq_fill(ctypes.Structure):
    _fields_ = [("raw", ctypes.c_void_p), ("n_samples", ctypes.c_int64),
                ("row_stride", ctypes.c_int64), ("n_channels", ctypes.c_int32),
                ("ped_samples", ctypes.c_int32), ("threshold", ctypes.c_int32),
                ("pre", ctypes.c_int32), ("post", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class daq_fill_out(ctypes.Structure):
    _fields_ = [("islands", ctypes.c_void_p), ("capacity", ctypes.c_int64),
                ("counts", ctypes.c_void_p), ("ped", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("out_stride", ctypes.c_int64)]


class daq_q_out(ctypes.Structure):
    _fields_ = [("qsum", ctypes.c_void_p), ("acc", ctypes.c_void_p), ("acc_stride", ctypes.c_int64),
                ("ped", ctypes.c_void_p)]


class daq_z_fill(ctypes.Structure):
    _fields_ = [("packed", ctypes.c_void_p), ("stride", ctypes.c_int64), ("counts", ctypes.c_void_p),
                ("max_len", ctypes.c_int64), ("hdr", ctypes.c_void_p), ("offsets", ctypes.c_void_p),
                ("words", ctypes.c_void_p), ("words_cap", ctypes.c_int64), ("n_words", ctypes.c_void_p),
                ("n_channels", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class daq_z_stream(ctypes.Structure):
    _fields_ = [("hdr", ctypes.c_void_p), ("offsets", ctypes.c_void_p), ("words", ctypes.c_void_p),
                ("n_words", ctypes.c_int64), ("out", ctypes.c_void_p), ("out_stride", ctypes.c_int64),
                ("n_samples", ctypes.c_int64), ("n_channels", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class daq_schedule(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_int32), ("wgs_per_cu", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("parts", ctypes.c_int32)]


class daq_counts(ctypes.Structure):
    _fields_ = [("n_islands", ctypes.c_int64), ("total_len", ctypes.c_int64),
                ("status", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class daq_completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("ticket", ctypes.c_uint64), ("counts", daq_counts),
                ("out", daq_fill_out), ("raw", ctypes.c_void_p), ("status", ctypes.c_int32),
                ("batch_fills", ctypes.c_int32), ("t_submit_ns", ctypes.c_int64),
                ("t_launch_ns", ctypes.c_int64), ("t_ready_ns", ctypes.c_int64)]


class daq_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("released", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("arena_bytes", ctypes.c_uint64),
                ("arena_in_use", ctypes.c_uint64), ("arena_peak", ctypes.c_uint64),
                ("pending", ctypes.c_int32), ("running", ctypes.c_int32),
                ("late", ctypes.c_uint64), ("timed_out", ctypes.c_uint64),
                ("deadtime_ns", ctypes.c_uint64), ("admit_wait_max_ns", ctypes.c_uint64)]


DAQ_SUBMIT_HOST_RAW = 1
DAQ_SUBMIT_HOST_PACKED12 = 2


class DaqError(RuntimeError):
    def __init__(self, code: int, where: str):
        lib = _lib_or_none()
        msg = lib.daq_strerror(code).decode() if lib else str(code)
        extra = ""
        if lib is not None and code == DAQ_EHIP:
            extra = " (hip error %d)" % lib.daq_last_hip_error()
        super().__init__("%s failed: %s%s" % (where, msg, extra))
        self.code = code


_lib = None


def _lib_or_none():
    return _lib


def load_library():
    """Loads libdaqisland.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libdaqisland.so is not built (run __graft_entry__.build() or "
                          "python paper_1611_04959_amd/build.py); there is no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "daq_version": ([], ctypes.c_char_p),
        "daq_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "daq_last_hip_error": ([], ctypes.c_int),
        "daq_max_islands": ([i64, i32, i32], i64),
        "daq_ctx_create": ([ctypes.POINTER(vp), ctypes.c_int], ctypes.c_int),
        "daq_ctx_destroy": ([vp], None),
        "daq_find_islands": ([vp, ctypes.POINTER(daq_fill), vp, i64, vp, vp, vp], ctypes.c_int),
        "daq_gather_islands": ([vp, ctypes.POINTER(daq_fill), vp, i64, vp, vp, i64, vp], ctypes.c_int),
        "daq_chop_fill": ([vp, ctypes.POINTER(daq_fill), ctypes.POINTER(daq_fill_out), vp], ctypes.c_int),
        "daq_process_batch": ([vp, ctypes.POINTER(daq_fill), ctypes.POINTER(daq_fill_out), i32, vp],
                              ctypes.c_int),
        "daq_process_batch_noalloc": ([vp, ctypes.POINTER(daq_fill), ctypes.POINTER(daq_fill_out), i32, vp],
                                      ctypes.c_int),
        "daq_noalloc_scratch_bytes": ([ctypes.POINTER(daq_fill), i32], i64),
        "daq_qmethod_batch": ([vp, ctypes.POINTER(daq_fill), ctypes.POINTER(daq_q_out), i32, vp],
                              ctypes.c_int),
        "daq_unpack12": ([vp, vp, i64, i32, i64, vp, i64, vp], ctypes.c_int),
        "daq_process_batch_q": ([vp, ctypes.POINTER(daq_fill), ctypes.POINTER(daq_fill_out),
                                 ctypes.POINTER(daq_q_out), i32, vp], ctypes.c_int),
        "daq_compress_batch": ([vp, ctypes.POINTER(daq_z_fill), i32, vp], ctypes.c_int),
        "daq_decompress_batch": ([vp, ctypes.POINTER(daq_z_stream), i32, vp], ctypes.c_int),
        "daq_packed12_stride": ([i64], i64),
        "daq_read_stream": ([vp, i64, vp, i32, i32, vp], ctypes.c_int),
        "daq_read_tiles": ([vp, i32, i32, i64, vp, i32, i32, vp, vp], ctypes.c_int),
        "daq_ctx_set_schedule": ([vp, ctypes.POINTER(daq_schedule)], ctypes.c_int),
        "daq_ctx_get_schedule": ([vp, ctypes.POINTER(daq_schedule)], ctypes.c_int),
        "daq_ctx_set_graphs": ([vp, ctypes.c_int], ctypes.c_int),
        "daq_ctx_get_graphs": ([vp, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "daq_ctx_set_timing": ([vp, ctypes.c_int], ctypes.c_int),
        "daq_ctx_kernel_time": ([vp, ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
        "daq_ctx_kernel_times": ([vp, ctypes.POINTER(ctypes.c_float), i32], ctypes.c_int),
        "daq_autotune": ([vp, ctypes.POINTER(daq_fill), ctypes.POINTER(daq_fill_out), i32, vp,
                          ctypes.c_char_p, ctypes.POINTER(daq_schedule)], ctypes.c_int),
        "daq_ctx_get_device": ([vp, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "daq_server_slot_bytes": ([ctypes.POINTER(daq_fill), i32, ctypes.POINTER(ctypes.c_uint64)],
                                  ctypes.c_int),
        "daq_server_create": ([ctypes.POINTER(vp), vp, vp, ctypes.c_size_t, i32, i32], ctypes.c_int),
        "daq_submit_fill": ([vp, ctypes.POINTER(daq_fill), i32, ctypes.c_uint64,
                             ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
        "daq_submit_fill_at": ([vp, ctypes.POINTER(daq_fill), i32, ctypes.c_uint64, i64,
                                ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
        "daq_server_set_limits": ([vp, i64, i64], ctypes.c_int),
        "daq_poll": ([vp, ctypes.POINTER(daq_completion), i32, i32], ctypes.c_int),
        "daq_release": ([vp, ctypes.c_uint64], ctypes.c_int),
        "daq_server_get_stats": ([vp, ctypes.POINTER(daq_server_stats)], ctypes.c_int),
        "daq_server_destroy": ([vp], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc: int, where: str):
    if rc != DAQ_OK:
        raise DaqError(rc, where)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream or None


def daq_max_islands(n_samples: int, pre: int, post: int) -> int:
    return int(load_library().daq_max_islands(n_samples, pre, post))


DAQ_NOALLOC_SCRATCH_BYTES = 32 << 20


def noalloc_scratch_bytes(fills: Sequence["Fill"]) -> int:
    """Scratch bytes daq_process_batch_noalloc needs for these fills (negative: an error code)."""
    n = len(fills)
    fa = (daq_fill * max(n, 1))()
    for i, f in enumerate(fills):
        fa[i] = f.c_struct()
    return int(load_library().daq_noalloc_scratch_bytes(fa, n))


def padded(n: int) -> int:
    return (int(n) + 7) // 8 * 8


@dataclasses.dataclass
class Fill:
    """One calorimeter fill on the device and its chopping parameters."""
    raw: object                 # torch.int16 [C, row_stride] (row_stride % 8 == 0)
    n_samples: int
    threshold: int = -200
    pre: int = 8
    post: int = 24
    ped_samples: int = 100

    def c_struct(self) -> daq_fill:
        r = self.raw
        if r.dim() != 2 or r.stride(1) != 1:
            raise ValueError("raw must be a 2-D tensor with contiguous rows")
        return daq_fill(r.data_ptr(), int(self.n_samples), int(r.stride(0)), int(r.shape[0]),
                        int(self.ped_samples), int(self.threshold), int(self.pre), int(self.post), 0)


@dataclasses.dataclass
class FillOut:
    """Device buffers for one fill's results."""
    islands: object             # torch.int64 [capacity, 3]
    counts: object              # torch.int64 [3]
    ped: object = None          # torch.int32 [C] or None
    out: object = None          # torch.int16 [C, out_stride] or None

    def c_struct(self) -> daq_fill_out:
        cap = int(self.islands.shape[0]) if self.islands is not None else 0
        ost = int(self.out.stride(0)) if self.out is not None else 0
        return daq_fill_out(_ptr(self.islands), cap, _ptr(self.counts), _ptr(self.ped),
                            _ptr(self.out), ost)

    def host(self):
        """Copies the results back: (islands[n], n_islands, total_len, status, ped, out[:, :total])."""
        cnt = self.counts.cpu().numpy()
        n, total, status = int(cnt[0]), int(cnt[1]), int(cnt[2]) & 0xFFFFFFFF
        isl = self.islands[:min(n, self.islands.shape[0])].cpu().numpy()
        ped = self.ped.cpu().numpy() if self.ped is not None else None
        out = None
        if self.out is not None:
            out = self.out[:, :min(total, self.out.shape[1])].cpu().numpy()
        return isl, n, total, status, ped, out


def alloc_out(fill: Fill, capacity: Optional[int] = None, gather: bool = True,
              device=None) -> FillOut:
    """Output buffers that can never overflow (capacity = daq_max_islands)."""
    import torch
    dev = device or fill.raw.device
    C = int(fill.raw.shape[0])
    cap = daq_max_islands(fill.n_samples, fill.pre, fill.post) if capacity is None else capacity
    isl = torch.empty((max(cap, 0), 3), dtype=torch.int64, device=dev)
    counts = torch.zeros(3, dtype=torch.int64, device=dev)
    ped = torch.empty(C, dtype=torch.int32, device=dev)
    out = torch.empty((C, max(padded(fill.n_samples), 8)), dtype=torch.int16, device=dev) if gather else None
    return FillOut(isl, counts, ped, out)


DAQ_Q_DECIMATION = 32


@dataclasses.dataclass
class QOut:
    """Device buffers of one fill's Q-method results (any may be None)."""
    qsum: object = None         # torch.int64 [ceil(N / 32)]
    acc: object = None          # torch.int32 [C, acc_stride] (acc_stride % 4 == 0), updated in place
    ped: object = None          # torch.int32 [C]

    def c_struct(self) -> daq_q_out:
        ast = int(self.acc.stride(0)) if self.acc is not None else 0
        return daq_q_out(_ptr(self.qsum), _ptr(self.acc), ast, _ptr(self.ped))


def alloc_q_out(fill: Fill, acc: bool = True, qsum: bool = True, device=None) -> QOut:
    """Q-method buffers for one fill; the accumulator starts at zero."""
    import torch
    dev = device or fill.raw.device
    C = int(fill.raw.shape[0])
    nb = (int(fill.n_samples) + DAQ_Q_DECIMATION - 1) // DAQ_Q_DECIMATION
    q = torch.zeros(max(nb, 1), dtype=torch.int64, device=dev) if qsum else None
    a = torch.zeros((C, max(padded(fill.n_samples), 8)), dtype=torch.int32, device=dev) if acc else None
    return QOut(q, a, torch.zeros(C, dtype=torch.int32, device=dev))


DAQ_Z_BLOCK = 64
DAQ_Z_MAX_WIDTH = 17


@dataclasses.dataclass
class ZOut:
    """Device buffers of one fill's compressed stream."""
    hdr: object                 # torch.int32 [C * ceil(max_len / 64)] (uint32 bit patterns)
    offsets: object             # torch.int64 [same], or None
    words: object               # torch.int32 [words_cap] (uint32 bit patterns)
    n_words: object             # torch.int64 [1]

    def host(self, n_channels: int, total_len: int):
        """(hdr, offsets, words) of a finished call as numpy uint32 / int64 arrays."""
        import numpy as np
        nb = (int(total_len) + DAQ_Z_BLOCK - 1) // DAQ_Z_BLOCK * int(n_channels)
        nw = int(self.n_words.item())
        hdr = self.hdr[:nb].cpu().numpy().view(np.uint32)
        offs = self.offsets[:nb].cpu().numpy() if self.offsets is not None else None
        words = self.words[:min(nw, int(self.words.numel()))].cpu().numpy().view(np.uint32)
        return hdr, offs, words


def z_words_bound(n_channels: int, max_len: int) -> int:
    """Words a stream of n_channels rows of at most max_len samples can need."""
    nb = (int(max_len) + DAQ_Z_BLOCK - 1) // DAQ_Z_BLOCK
    return int(n_channels) * nb * 34


def alloc_z_out(n_channels: int, max_len: int, words_cap: Optional[int] = None, offsets: bool = True,
                device=None) -> ZOut:
    """Buffers for one fill's stream; the default words_cap never cuts it short."""
    import torch
    nb = (int(max_len) + DAQ_Z_BLOCK - 1) // DAQ_Z_BLOCK * int(n_channels)
    cap = z_words_bound(n_channels, max_len) if words_cap is None else int(words_cap)
    return ZOut(torch.zeros(max(nb, 1), dtype=torch.int32, device=device),
                torch.zeros(max(nb, 1), dtype=torch.int64, device=device) if offsets else None,
                torch.zeros(max(cap, 1), dtype=torch.int32, device=device),
                torch.zeros(1, dtype=torch.int64, device=device))


class Batch:
    """The C arrays of one batch (daq_fill and daq_fill_out per fill), built
    once so that repeated launches of the same fills and outputs skip the
    argument marshalling. Holds references to the fills and outputs."""

    def __init__(self, fills: Sequence["Fill"], outs: Sequence["FillOut"]):
        if len(fills) != len(outs):
            raise ValueError("fills and outs differ in length")
        self.fills, self.outs = list(fills), list(outs)
        self.n = len(self.fills)
        self.fa = (daq_fill * max(self.n, 1))()
        self.oa = (daq_fill_out * max(self.n, 1))()
        for i, (f, o) in enumerate(zip(self.fills, self.outs)):
            self.fa[i] = f.c_struct()
            self.oa[i] = o.c_struct()


class Context:
    """A daq_ctx on one HIP device."""

    def __init__(self, device: int = 0):
        self._lib = load_library()
        h = ctypes.c_void_p()
        _check(self._lib.daq_ctx_create(ctypes.byref(h), int(device)), "daq_ctx_create")
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            self._lib.daq_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- the C calls -----------------------------------------------------
    def daq_find_islands(self, fill: Fill, fo: FillOut, stream=None):
        cap = int(fo.islands.shape[0]) if fo.islands is not None else 0
        f = fill.c_struct()
        _check(self._lib.daq_find_islands(self.handle, ctypes.byref(f), _ptr(fo.islands), cap,
                                          _ptr(fo.counts), _ptr(fo.ped), _stream_handle(stream)),
               "daq_find_islands")

    def daq_gather_islands(self, fill: Fill, fo: FillOut, stream=None):
        cap = int(fo.islands.shape[0]) if fo.islands is not None else 0
        f = fill.c_struct()
        _check(self._lib.daq_gather_islands(self.handle, ctypes.byref(f), _ptr(fo.islands), cap,
                                            _ptr(fo.counts), _ptr(fo.out),
                                            int(fo.out.stride(0)) if fo.out is not None else 0,
                                            _stream_handle(stream)),
               "daq_gather_islands")

    def daq_chop_fill(self, fill: Fill, fo: FillOut, stream=None):
        f = fill.c_struct()
        o = fo.c_struct()
        _check(self._lib.daq_chop_fill(self.handle, ctypes.byref(f), ctypes.byref(o),
                                       _stream_handle(stream)), "daq_chop_fill")

    def _arrays(self, fills: Sequence[Fill], outs: Sequence[FillOut]):
        if len(fills) != len(outs):
            raise ValueError("fills and outs differ in length")
        n = len(fills)
        fa = (daq_fill * max(n, 1))()
        oa = (daq_fill_out * max(n, 1))()
        for i, (f, o) in enumerate(zip(fills, outs)):
            fa[i] = f.c_struct()
            oa[i] = o.c_struct()
        return fa, oa, n

    def daq_process_batch(self, fills, outs: Optional[Sequence[FillOut]] = None, stream=None):
        """fills: a sequence of Fill (with outs), or a prepared Batch (outs None)."""
        if isinstance(fills, Batch):
            fa, oa, n = fills.fa, fills.oa, fills.n
        else:
            fa, oa, n = self._arrays(fills, outs)
        _check(self._lib.daq_process_batch(self.handle, fa, oa, n, _stream_handle(stream)),
               "daq_process_batch")

    def daq_process_batch_noalloc(self, fills: Sequence[Fill], outs: Sequence[FillOut], stream=None):
        """daq_process_batch without any allocation (scratch in the library's static device array)."""
        fa, oa, n = self._arrays(fills, outs)
        _check(self._lib.daq_process_batch_noalloc(self.handle, fa, oa, n, _stream_handle(stream)),
               "daq_process_batch_noalloc")

    def daq_qmethod_batch(self, fills: Sequence[Fill], qouts: Sequence[QOut], stream=None):
        if len(fills) != len(qouts):
            raise ValueError("fills and qouts differ in length")
        n = len(fills)
        fa = (daq_fill * max(n, 1))()
        qa = (daq_q_out * max(n, 1))()
        for i, (f, q) in enumerate(zip(fills, qouts)):
            fa[i] = f.c_struct()
            qa[i] = q.c_struct()
        _check(self._lib.daq_qmethod_batch(self.handle, fa, qa, n, _stream_handle(stream)),
               "daq_qmethod_batch")

    def daq_process_batch_q(self, fills: Sequence[Fill], outs: Sequence[FillOut], qouts: Sequence[QOut],
                            stream=None):
        """The T-method (outs) and the Q-method (qouts) on one read of the raw samples."""
        fa, oa, n = self._arrays(fills, outs)
        if len(qouts) != n:
            raise ValueError("fills and qouts differ in length")
        qa = (daq_q_out * max(n, 1))()
        for i, q in enumerate(qouts):
            qa[i] = q.c_struct()
        _check(self._lib.daq_process_batch_q(self.handle, fa, oa, qa, n, _stream_handle(stream)),
               "daq_process_batch_q")

    def daq_unpack12(self, packed, n_samples: int, raw, stream=None):
        """packed: uint8 [C, packed_stride] on the device; raw: int16 [C, row_stride] (written)."""
        _check(self._lib.daq_unpack12(self.handle, packed.data_ptr(), int(packed.stride(0)), int(packed.shape[0]),
                                      int(n_samples), raw.data_ptr(), int(raw.stride(0)), _stream_handle(stream)),
               "daq_unpack12")

    def daq_compress_batch(self, outs: Sequence[FillOut], zouts: Sequence[ZOut], max_len: Optional[int] = None,
                           words_cap: Optional[Sequence[int]] = None, stream=None):
        """Compress the packed rows of each chopped fill (outs[i].out, total_len from outs[i].counts)."""
        if len(outs) != len(zouts):
            raise ValueError("outs and zouts differ in length")
        n = len(outs)
        za = (daq_z_fill * max(n, 1))()
        for i, (o, z) in enumerate(zip(outs, zouts)):
            ml = int(o.out.shape[1]) if max_len is None else int(max_len)
            cap = int(z.words.numel()) if words_cap is None else int(words_cap[i])
            za[i] = daq_z_fill(o.out.data_ptr(), int(o.out.stride(0)), o.counts.data_ptr(), ml, z.hdr.data_ptr(),
                               _ptr(z.offsets), z.words.data_ptr(), cap, z.n_words.data_ptr(),
                               int(o.out.shape[0]), 0)
        _check(self._lib.daq_compress_batch(self.handle, za, n, _stream_handle(stream)), "daq_compress_batch")

    def daq_decompress_batch(self, zouts: Sequence[ZOut], n_samples: Sequence[int], outs, stream=None):
        """Decode streams made by daq_compress_batch (n_samples: each stream's total_len) into
        int16 [C, out_stride] tensors `outs`."""
        if not (len(zouts) == len(n_samples) == len(outs)):
            raise ValueError("zouts, n_samples and outs differ in length")
        n = len(zouts)
        za = (daq_z_stream * max(n, 1))()
        for i, (z, L, o) in enumerate(zip(zouts, n_samples, outs)):
            if z.offsets is None:
                raise ValueError("decoding needs the block offsets")
            # the words the buffer holds bound the reads (no device round trip per call)
            za[i] = daq_z_stream(z.hdr.data_ptr(), z.offsets.data_ptr(), z.words.data_ptr(),
                                 int(z.words.numel()), o.data_ptr(), int(o.stride(0)), int(L),
                                 int(o.shape[0]), 0)
        _check(self._lib.daq_decompress_batch(self.handle, za, n, _stream_handle(stream)),
               "daq_decompress_batch")

    def daq_autotune(self, fills: Sequence[Fill], outs: Sequence[FillOut], stream=None,
                     cache_path: Optional[str] = None) -> daq_schedule:
        fa, oa, n = self._arrays(fills, outs)
        best = daq_schedule()
        _check(self._lib.daq_autotune(self.handle, fa, oa, n, _stream_handle(stream),
                                      cache_path.encode() if cache_path else None,
                                      ctypes.byref(best)), "daq_autotune")
        return best

    # -- settings ----------------------------------------------------------
    def set_schedule(self, threads: int = 256, wgs_per_cu: int = 16, variant: int = 5, parts: int = 0):
        s = daq_schedule(threads, wgs_per_cu, variant, parts)
        _check(self._lib.daq_ctx_set_schedule(self.handle, ctypes.byref(s)), "daq_ctx_set_schedule")

    def get_schedule(self) -> daq_schedule:
        s = daq_schedule()
        _check(self._lib.daq_ctx_get_schedule(self.handle, ctypes.byref(s)), "daq_ctx_get_schedule")
        return s

    def set_graphs(self, enable: bool):
        _check(self._lib.daq_ctx_set_graphs(self.handle, int(bool(enable))), "daq_ctx_set_graphs")

    def get_graphs(self) -> bool:
        v = ctypes.c_int(0)
        _check(self._lib.daq_ctx_get_graphs(self.handle, ctypes.byref(v)), "daq_ctx_get_graphs")
        return bool(v.value)

    def set_timing(self, enable: bool):
        _check(self._lib.daq_ctx_set_timing(self.handle, int(bool(enable))), "daq_ctx_set_timing")

    def kernel_times_ms(self, max_n: int = 1 << 14) -> List[float]:
        buf = (ctypes.c_float * max_n)()
        n = self._lib.daq_ctx_kernel_times(self.handle, buf, max_n)
        if n < 0:
            _check(n, "daq_ctx_kernel_times")
        return [float(buf[i]) for i in range(n)]

    def kernel_time_ms(self) -> float:
        ms = ctypes.c_float()
        _check(self._lib.daq_ctx_kernel_time(self.handle, ctypes.byref(ms)), "daq_ctx_kernel_time")
        return float(ms.value)


def read_stream(buf, sink, blocks: int, layout: int = 0, stream=None):
    """daq_read_stream: one streaming read of a device tensor (the device's read ceiling)."""
    if sink.numel() * sink.element_size() < 4 * 4 * int(blocks):
        raise ValueError("the sink holds one 32-bit word per wave: %d words" % (4 * int(blocks)))
    _check(load_library().daq_read_stream(buf.data_ptr(), int(buf.numel() * buf.element_size()),
                                          sink.data_ptr(), int(blocks), int(layout), _stream_handle(stream)),
           "daq_read_stream")


def read_tiles(raw, n_fills: int, channels: int, n_samples: int, sink, blocks: int, mode: int = 0, out=None,
               stream=None):
    """daq_read_tiles: the chop scan's read pattern over n_fills fills stored
    back to back in the int16 device tensor `raw` (mode 0), plus the re-read
    (mode 1) and the re-read and packed write (mode 2, into `out`) of a fixed
    island pattern."""
    import torch
    if raw.dtype != torch.int16 or raw.numel() < int(n_fills) * int(channels) * int(n_samples):
        raise ValueError("raw must be int16 holding n_fills x channels x n_samples samples")
    if sink.numel() * sink.element_size() < 4 * 8 * int(blocks):
        raise ValueError("the sink holds one 32-bit word per wave: %d words" % (8 * int(blocks)))
    out_ptr = None
    if int(mode) == 2:
        tiles = (int(n_samples) + 4047) // 4048
        need = int(n_fills) * tiles * int(channels) * 512 * 16
        if out is None or out.numel() * out.element_size() < need:
            raise ValueError("mode 2 writes %d bytes to out" % need)
        out_ptr = out.data_ptr()
    _check(load_library().daq_read_tiles(raw.data_ptr(), int(n_fills), int(channels), int(n_samples),
                                         sink.data_ptr(), int(blocks), int(mode), out_ptr,
                                         _stream_handle(stream)),
           "daq_read_tiles")


def version() -> str:
    return load_library().daq_version().decode()


__all__: List[str] = ["Batch", "Context", "Fill", "FillOut", "alloc_out", "ZOut", "alloc_z_out", "z_words_bound", "daq_max_islands", "load_library",
                      "version", "DaqError", "padded", "daq_schedule"]


def slot_bytes(fill: Fill, host_raw: bool = False, host_packed12: bool = False) -> int:
    """Arena bytes one fill's slot takes in a Server (daq_server_slot_bytes)."""
    lib = load_library()
    b = ctypes.c_uint64(0)
    f = fill.c_struct()
    flags = (DAQ_SUBMIT_HOST_RAW if host_raw else 0) | (DAQ_SUBMIT_HOST_PACKED12 if host_packed12 else 0)
    _check(lib.daq_server_slot_bytes(ctypes.byref(f), flags, ctypes.byref(b)), "daq_server_slot_bytes")
    return int(b.value)


def packed12_stride(n_samples: int) -> int:
    """Bytes per channel row of a fill submitted as 12-bit words (daq_packed12_stride)."""
    return int(load_library().daq_packed12_stride(int(n_samples)))


@dataclasses.dataclass
class Completion:
    """A finished fill (daq_completion) and where its results sit in the arena."""
    tag: int
    ticket: int
    n_islands: int
    total_len: int
    status: int
    error: int
    batch_fills: int
    t_submit_ns: int
    t_launch_ns: int
    t_ready_ns: int
    islands_ptr: int
    capacity: int
    ped_ptr: int
    out_ptr: int
    out_stride: int

    @property
    def latency_ms(self) -> float:
        return (self.t_ready_ns - self.t_submit_ns) * 1e-6


class Server:
    """daq_server: admission by HBM budget and continuous batching.

    ``arena`` is a device ``torch.uint8`` tensor (the budget); it must outlive
    the server. ``Context`` supplies the device and the kernel schedule.
    """

    def __init__(self, ctx: Context, arena, n_streams: int = 2, max_batch: int = 16):
        self._lib = load_library()
        self.arena = arena
        self._base = int(arena.data_ptr())
        h = ctypes.c_void_p()
        _check(self._lib.daq_server_create(ctypes.byref(h), ctx.handle, self._base, int(arena.numel()),
                                           int(n_streams), int(max_batch)), "daq_server_create")
        self._h = h
        self._buf = (daq_completion * 256)()

    def close(self):
        if getattr(self, "_h", None):
            self._lib.daq_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_limits(self, admit_deadline_us: int = 10_000, batch_timeout_us: int = 10_000_000):
        """daq_server_set_limits: admission deadline (late fills) and batch time-out (watchdog)."""
        _check(self._lib.daq_server_set_limits(self._h, int(admit_deadline_us), int(batch_timeout_us)),
               "daq_server_set_limits")

    def submit(self, fill: Fill, tag: int = 0, host_raw=None, host_packed12=None,
               arrival_ns: int = 0) -> Optional[int]:
        """Admits a fill; returns its ticket, or None when the budget is full now.

        ``arrival_ns`` (``time.monotonic_ns()`` of the fill's arrival; 0 = now)
        lets a caller that retries after a refusal keep the first attempt's
        time (daq_submit_fill_at).

        With ``host_raw`` (a CPU int16 [C, row_stride] tensor, pinned for
        speed) the samples are copied into the arena by the server and
        ``fill.raw`` is only used for its shape. With ``host_packed12`` (a
        CPU uint8 [C, packed12_stride(N)] tensor of 12-bit words) the words
        are copied and unpacked on the device; ``fill.raw`` gives the shape
        (channels, row stride)."""
        f = fill.c_struct()
        flags = 0
        if host_packed12 is not None:
            if host_raw is not None:
                raise ValueError("host_raw and host_packed12 exclude each other")
            N = int(fill.n_samples)
            if (host_packed12.dim() != 2 or host_packed12.is_cuda or host_packed12.dtype.itemsize != 1
                    or host_packed12.shape[0] != f.n_channels
                    or host_packed12.stride(0) != packed12_stride(N) or host_packed12.stride(1) != 1):
                raise ValueError("host_packed12 must be a CPU uint8 [C, packed12_stride(N)] tensor")
            f.raw = host_packed12.data_ptr()
            flags = DAQ_SUBMIT_HOST_PACKED12
        if host_raw is not None:
            if host_raw.dim() != 2 or host_raw.stride(1) != 1 or host_raw.is_cuda:
                raise ValueError("host_raw must be a 2-D CPU tensor with contiguous rows")
            f.raw = host_raw.data_ptr()
            f.row_stride = int(host_raw.stride(0))
            f.n_channels = int(host_raw.shape[0])
            flags = DAQ_SUBMIT_HOST_RAW
        t = ctypes.c_uint64(0)
        rc = self._lib.daq_submit_fill_at(self._h, ctypes.byref(f), flags, int(tag), int(arrival_ns),
                                          ctypes.byref(t))
        if rc == DAQ_EAGAIN:
            return None
        _check(rc, "daq_submit_fill")
        return int(t.value)

    def poll(self, max_n: int = 256, timeout_us: int = 0) -> List[Completion]:
        n = self._lib.daq_poll(self._h, self._buf, min(int(max_n), 256), int(timeout_us))
        if n < 0:
            _check(n, "daq_poll")
        res = []
        for i in range(n):
            c = self._buf[i]
            res.append(Completion(int(c.tag), int(c.ticket), int(c.counts.n_islands),
                                  int(c.counts.total_len), int(c.counts.status) & 0xFFFFFFFF,
                                  int(c.status), int(c.batch_fills), int(c.t_submit_ns),
                                  int(c.t_launch_ns), int(c.t_ready_ns), int(c.out.islands or 0),
                                  int(c.out.capacity), int(c.out.ped or 0), int(c.out.out or 0),
                                  int(c.out.out_stride)))
        return res

    def release(self, ticket: int):
        _check(self._lib.daq_release(self._h, int(ticket)), "daq_release")

    def try_release(self, ticket: int) -> int:
        return int(self._lib.daq_release(self._h, int(ticket)))

    def stats(self) -> daq_server_stats:
        st = daq_server_stats()
        _check(self._lib.daq_server_get_stats(self._h, ctypes.byref(st)), "daq_server_get_stats")
        return st

    # the C names
    daq_submit_fill = submit
    daq_poll = poll
    daq_release = release

    def results(self, c: Completion, n_channels: int):
        """Host copies of a completion's results: (islands[n], ped, out[:, :total_len])."""
        import torch
        a = self.arena

        def view(ptr, nbytes, dtype):
            off = ptr - self._base
            return a[off:off + nbytes].view(dtype)

        n = min(c.n_islands, c.capacity)
        isl = view(c.islands_ptr, n * 24, torch.int64).reshape(n, 3).cpu().numpy()
        ped = view(c.ped_ptr, 4 * n_channels, torch.int32).cpu().numpy()
        rows = view(c.out_ptr, 2 * n_channels * c.out_stride, torch.int16).reshape(n_channels, c.out_stride)
        out = rows[:, :min(c.total_len, c.out_stride)].cpu().numpy()
        return isl, ped, out
