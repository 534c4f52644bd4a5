"""Helpers for the GPU parity tests: run the HIP library through its C ABI
on device copies of host fills, and compare with the CPU oracle."""
import concurrent.futures as cf
import os

import numpy as np

import oracle
import paper_1611_04959_amd as daq


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
