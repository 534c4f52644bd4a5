"""Helpers for the GPU parity tests: run the HIP library through its C ABI
on device copies of host fills, and compare with the CPU oracle.

Every output buffer a GPU test hands to the library is filled with a poison
pattern first (and again before every call made through ``run``): a kernel
that leaves a record field, a pedestal, a count or a packed sample unwritten
then fails the comparison, instead of passing on values that an earlier call
left in memory the caching allocator handed out again. Importing this module
installs poisoning versions of the binding's ``alloc_out``, ``alloc_q_out``
and ``alloc_z_out``.
"""
import concurrent.futures as cf
import os

import numpy as np

import oracle
import paper_1611_04959_amd as daq

#: poison byte of sample, pedestal, sum and stream buffers; record and count
#: buffers get 0xFF (every field reads -1, an impossible value)
POISON = 0x5A
POISON_REC = 0xFF


def poison(t, byte=POISON):
    """Fills a device tensor's bytes with `byte` (no-op for None / empty)."""
    import torch
    if t is None or t.numel() == 0:
        return t
    if t.is_contiguous():
        t.view(-1).view(torch.uint8).fill_(byte)
    else:
        t.fill_(int.from_bytes(bytes([byte]) * t.element_size(), "little", signed=t.is_signed()))
    return t


def poison_out(o):
    """Poisons every output buffer of a FillOut."""
    poison(o.islands, POISON_REC)
    poison(o.counts, POISON_REC)
    poison(o.ped)
    poison(o.out)
    return o


def poison_q(q):
    """Poisons a QOut's written outputs (the accumulator keeps its contents:
    calls add into it)."""
    poison(q.qsum)
    poison(q.ped)
    return q


def poison_z(z):
    poison(z.hdr)
    poison(z.offsets, POISON_REC)
    poison(z.words)
    poison(z.n_words, POISON_REC)
    return z


_alloc_out, _alloc_q_out, _alloc_z_out = daq.alloc_out, daq.alloc_q_out, daq.alloc_z_out


def _alloc_out_poisoned(*a, **k):
    return poison_out(_alloc_out(*a, **k))


def _alloc_q_out_poisoned(*a, **k):
    return poison_q(_alloc_q_out(*a, **k))


def _alloc_z_out_poisoned(*a, **k):
    return poison_z(_alloc_z_out(*a, **k))


if not getattr(daq.alloc_out, "poisoned", False):
    _alloc_out_poisoned.poisoned = True
    daq.alloc_out = _alloc_out_poisoned
    daq.alloc_q_out = _alloc_q_out_poisoned
    daq.alloc_z_out = _alloc_z_out_poisoned


def poison_slot(srv, c, n_channels):
    """Poisons the arena regions of a served completion (records, pedestals,
    packed rows) so that the slot's next user starts from poison."""
    a = srv.arena
    base = srv._base

    def region(ptr, nbytes, byte):
        if ptr and nbytes > 0:
            a[ptr - base:ptr - base + nbytes].fill_(byte)

    region(c.islands_ptr, 24 * c.capacity, POISON_REC)
    region(c.ped_ptr, 4 * n_channels, POISON)
    region(c.out_ptr, 2 * n_channels * c.out_stride, POISON)


def log(msg):
    print("[gpu-test] " + msg, flush=True)


def pad_stride(x):
    """int16 [C, N] -> [C, padded(N)] zero padded (row stride % 8 == 0)."""
    C, N = x.shape
    st = max(daq.padded(N), 8)
    y = np.zeros((C, st), np.int16)
    y[:, :N] = x
    return y


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def make_fill(xd, n, p):
    return daq.Fill(xd, n, threshold=p["threshold"], pre=p["pre"], post=p["post"],
                    ped_samples=p["ped_samples"])


def oracle_result(x, n, p, capacity=None):
    return oracle.chop(x, n_samples=n, ped_samples=p["ped_samples"], threshold=p["threshold"],
                       pre=p["pre"], post=p["post"], capacity=capacity)


def oracle_many(xs, ns, ps):
    workers = min(16, os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(workers) as ex:
        return list(ex.map(lambda a: oracle_result(*a), zip(xs, ns, ps)))


def assert_same(fo, ref, ctx="", out_check=True):
    isl, n, total, status, ped, out = fo.host()
    assert n == ref.n_islands, "%s: n_islands %d != %d" % (ctx, n, ref.n_islands)
    assert total == ref.total_len, "%s: total_len %d != %d" % (ctx, total, ref.total_len)
    assert status == 0, "%s: status %d" % (ctx, status)
    np.testing.assert_array_equal(ped, ref.ped, err_msg=ctx + ": pedestals")
    np.testing.assert_array_equal(isl, ref.islands, err_msg=ctx + ": island records")
    if out_check and fo.out is not None:
        np.testing.assert_array_equal(out, ref.out, err_msg=ctx + ": packed samples")


def run(ctx, mode, fills, outs, stream=None):
    """mode: 'chop' (fused, per fill), 'twopass' (find + gather per fill), 'batch'."""
    import torch
    for o in outs:
        poison_out(o)
    if mode == "chop":
        for f, o in zip(fills, outs):
            ctx.daq_chop_fill(f, o, stream)
    elif mode == "twopass":
        for f, o in zip(fills, outs):
            ctx.daq_find_islands(f, o, stream)
            ctx.daq_gather_islands(f, o, stream)
    elif mode == "batch":
        ctx.daq_process_batch(fills, outs, stream)
    else:
        raise ValueError(mode)
    torch.cuda.synchronize()
