"""HBM traffic of the chop pass from rocprofv3 counters.

Two counter runs of the benchmark (``FETCH_SIZE``, then ``WRITE_SIZE``, in
KiB per dispatch) give the bytes each kernel moved between L2 and memory.
The counters are scaled by what they read for a plain copy of known size
(``python -m paper_1611_04959_amd.traffic copy``, torch's copy kernel), so
the reported figures are bytes.

  python -m paper_1611_04959_amd.traffic copy [MiB]
  python -m paper_1611_04959_amd.traffic summarize FETCH_DIR WRITE_DIR \
         COPY_FETCH_DIR COPY_WRITE_DIR OUT_JSON [fills]
  python -m paper_1611_04959_amd.traffic stats KERNEL_STATS_CSV

  python -m paper_1611_04959_amd.traffic tail KERNEL_TRACE_CSV K
  python -m paper_1611_04959_amd.traffic streams KERNEL_TRACE_CSV K

``summarize`` writes OUT_JSON (read by bench.py) and prints a text summary;
``stats`` prints a rocprofv3 ``--stats`` kernel table as markdown; ``tail``
prints the mean duration of each chop kernel over its last K dispatches and
the mean span of the last K launches (first kernel start to last kernel end),
i.e. the timed steps of a run whose autotuning came first; ``streams`` does
the same for launches that alternate over several streams, with the span of
all K and the share of it during which two or more streams ran kernels.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
#: the sources of the chop kernels (the kernels and their shared internal
#: header): the counts recorded for one version are not reported for another
KERNEL_SOURCES = (os.path.join(HERE, "csrc", "chop_kernels.hip"), os.path.join(HERE, "csrc", "chop_internal.h"))
PASS_KERNELS = ("k_prepare", "k_scan_pass", "k_edge_pass", "k_copy_pass", "k_chop", "k_pipe")


def _code_only(text: str) -> str:
    """The source without comments and with runs of white space collapsed:
    what the compiler sees, so that a comment edit keeps the counts valid.
    (String literals in these sources hold no comment markers.)"""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_sha() -> str:
    """Hash of the code (comments and spacing aside) of every source the chop
    kernels are built from."""
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        h.update(os.path.basename(path).encode() + b"\0")
        h.update(_code_only(open(path, encoding="utf-8").read()).encode())
    return h.hexdigest()[:16]


def copy_run(mib: int = 1024, reps: int = 3):
    import torch
    n = mib * (1 << 20) // 2
    src = torch.ones(n, dtype=torch.int16, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print("copied %d x %d MiB" % (reps, mib), flush=True)


def _rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError("no counter_collection.csv under " + d)
    for f in files:
        with open(f, newline="") as fh:
            yield from csv.DictReader(fh)


def per_kernel(d, counter):
    """kernel short name -> list of per-dispatch counter values (KiB)."""
    acc = defaultdict(lambda: defaultdict(float))  # kernel -> dispatch -> value
    for r in _rows(d):
        if r.get("Counter_Name") != counter:
            continue
        name = r.get("Kernel_Name", "")
        acc[name][r.get("Dispatch_Id")] += float(r.get("Counter_Value", 0) or 0)
    return {k: list(v.values()) for k, v in acc.items()}


def short(name):
    for k in PASS_KERNELS:
        if k in name:
            return k
    return None


def copy_factor(d, counter, mib):
    vals = [v for k, vs in per_kernel(d, counter).items() if "copy" in k.lower() or "elementwise" in k
            for v in vs]
    vals = [v for v in vals if v > mib * 1024 * 0.5]  # the big copies only
    if not vals:
        raise RuntimeError("copy kernel not found in " + d)
    kib = sum(vals) / len(vals)
    return mib * (1 << 20) / (kib * 1024), kib


def summarize(fetch_dir, write_dir, cf_dir, cw_dir, out_json, fills=16, mib=1024):
    f_fac, f_kib = copy_factor(cf_dir, "FETCH_SIZE", mib)
    w_fac, w_kib = copy_factor(cw_dir, "WRITE_SIZE", mib)
    fetch = per_kernel(fetch_dir, "FETCH_SIZE")
    write = per_kernel(write_dir, "WRITE_SIZE")
    kern = {}
    for name, vs in fetch.items():
        k = short(name)
        if k is None or not vs:
            continue
        ws = write.get(name, [0.0])
        # every dispatch of these kernels is one 16-fill launch: take the median
        fk, wk = sorted(vs)[len(vs) // 2], sorted(ws)[len(ws) // 2]
        kern[k] = {"fetch_bytes": fk * 1024 * f_fac, "write_bytes": wk * 1024 * w_fac,
                   "dispatches": len(vs), "fetch_kib_raw": fk, "write_kib_raw": wk}
    # the timed launch: one graph of all the pass's kernels
    total = sum(v["fetch_bytes"] + v["write_bytes"] for v in kern.values())
    res = {"kernel_sha": kernel_sha(), "fills": fills, "bytes_per_launch": round(total),
           "copy_factor_fetch": f_fac, "copy_factor_write": w_fac,
           "copy_fetch_kib": f_kib, "copy_write_kib": w_kib, "copy_mib": mib, "kernels": kern}
    with open(out_json, "w") as fh:
        json.dump(res, fh, indent=1)
    print("copy calibration: %d MiB copy reads FETCH_SIZE %.0f KiB (x%.3f), WRITE_SIZE %.0f KiB (x%.3f)"
          % (mib, f_kib, f_fac, w_kib, w_fac))
    for k, v in sorted(kern.items()):
        print("%-14s fetch %10.1f MB  write %9.1f MB  (raw %.0f / %.0f KiB, %d dispatches)"
              % (k, v["fetch_bytes"] / 1e6, v["write_bytes"] / 1e6, v["fetch_kib_raw"], v["write_kib_raw"],
                 v["dispatches"]))
    print("per timed launch: %.1f MB" % (total / 1e6))
    return res


def stats_table(path):
    rows = list(csv.DictReader(open(path, newline="")))
    print("| Kernel | Calls | Average (us) | Min (us) | Max (us) | Share |")
    print("|---|---|---|---|---|---|")
    for r in rows:
        name = r["Name"].replace("daqk::(anonymous namespace)::", "").replace("void ", "")
        name = name if len(name) <= 60 else name[:57] + "..."
        print("| `%s` | %s | %.1f | %.1f | %.1f | %.1f %% |" % (
            name, r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
            float(r["Percentage"])))
    pas = [r for r in rows if any(k in r["Name"] for k in PASS_KERNELS)]
    tot = sum(float(r["AverageNs"]) for r in pas) / 1e3
    print()
    print("One launch (every kernel above named k_*): %.1f us of kernel time." % tot)


def tail(path, k):
    rows = list(csv.DictReader(open(path, newline="")))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    seq = []
    for r in rows:
        name = short(r["Kernel_Name"])
        if name is not None:
            seq.append((name, int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]))
    # launches: a scan (or fused) dispatch opens one; keep the last k
    opens = [i for i, x in enumerate(seq) if x[0] in ("k_scan_pass", "k_chop", "k_pipe")][-k:]
    if not opens:
        print("no launch found")
        return
    window = seq[opens[0]:]
    per = {}
    for name, a, b, full in window:
        per.setdefault(name, []).append((a, b, full))
    print("| Kernel | Dispatches in the last %d launches | Mean (us) |" % len(opens))
    print("|---|---|---|")
    for name, v in sorted(per.items(), key=lambda kv: kv[1][0][0]):
        t = [(b - a) / 1e3 for a, b, _ in v]
        label = v[-1][2].replace("daqk::(anonymous namespace)::", "").replace("void ", "").split("(")[0]
        print("| `%s` | %d | %.1f |" % (label, len(v), sum(t) / len(t)))
    spans = []
    for j, i in enumerate(opens):
        nxt = opens[j + 1] if j + 1 < len(opens) else len(seq)
        spans.append((seq[nxt - 1][2] - seq[i][1]) / 1e3)
    print()
    print("Mean span of the last %d launches (first kernel start to last kernel end): %.1f us"
          % (len(spans), sum(spans) / len(spans)))


def streams(path, k):
    """The last k launches of a run whose launches alternate over several
    streams: each chop kernel's mean duration, the launches per stream, the
    wall span from the first of those launches' start to the last kernel's
    end (and that span over k), and the share of the span during which
    kernels of two or more streams ran at once."""
    rows = list(csv.DictReader(open(path, newline="")))
    seq = []
    for r in rows:
        name = short(r["Kernel_Name"])
        if name is not None:
            seq.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), name, r.get("Stream_Id", "0")))
    seq.sort()
    opens = [i for i, x in enumerate(seq) if x[2] in ("k_scan_pass", "k_chop", "k_pipe")][-k:]
    if not opens:
        print("no launch found")
        return None
    window = seq[opens[0]:]
    per, by_stream = defaultdict(list), defaultdict(int)
    for a, b, name, sid in window:
        per[name].append((b - a) / 1e3)
        if name in ("k_scan_pass", "k_chop", "k_pipe"):
            by_stream[sid] += 1
    t0 = window[0][0]
    t1 = max(b for _, b, _, _ in window)
    # time with kernels of two or more streams in flight (sweep over edges)
    edges = sorted([(a, 1, sid) for a, _, _, sid in window] + [(b, -1, sid) for _, b, _, sid in window])
    live, both, last = defaultdict(int), 0, t0
    for t, d, sid in edges:
        if sum(1 for v in live.values() if v > 0) >= 2:
            both += t - last
        live[sid] += d
        last = t
    span = (t1 - t0) / 1e3
    print("| Kernel | Dispatches in the last %d launches | Mean (us) |" % len(opens))
    print("|---|---|---|")
    for name in ("k_prepare", "k_scan_pass", "k_edge_pass", "k_copy_pass", "k_chop", "k_pipe"):
        if name in per:
            print("| `%s` | %d | %.1f |" % (name, len(per[name]), sum(per[name]) / len(per[name])))
    print()
    print("Launches per stream: %s" % ", ".join("%s: %d" % kv for kv in sorted(by_stream.items())))
    print("Span of the last %d launches: %.1f us, %.1f us per launch; kernels of two or more streams "
          "in flight for %.0f %% of it" % (len(opens), span, span / len(opens), 100.0 * both / 1e3 / span))
    return {"span_us": span, "per_launch_us": span / len(opens), "overlap": both / 1e3 / span,
            "streams": dict(by_stream), "mean_us": {n: sum(v) / len(v) for n, v in per.items()}}


if __name__ == "__main__":
    if len(sys.argv) >= 2 and sys.argv[1] == "copy":
        copy_run(int(sys.argv[2]) if len(sys.argv) > 2 else 1024)
    elif len(sys.argv) == 3 and sys.argv[1] == "stats":
        stats_table(sys.argv[2])
    elif len(sys.argv) == 4 and sys.argv[1] == "tail":
        tail(sys.argv[2], int(sys.argv[3]))
    elif len(sys.argv) == 4 and sys.argv[1] == "streams":
        streams(sys.argv[2], int(sys.argv[3]))
    elif len(sys.argv) >= 7 and sys.argv[1] == "summarize":
        summarize(*sys.argv[2:7], fills=int(sys.argv[7]) if len(sys.argv) > 7 else 16)
    else:
        print(__doc__)
        sys.exit(2)
