"""Hardware-counter bookkeeping for the benchmark's roofline entry.

HBM traffic of a kernel launch is taken from two rocprofv3 counter runs of
``bench.py --counters P`` (one with FETCH_SIZE, one with WRITE_SIZE).  Both counters
report KiB per dispatch; on this hardware they do not count every memory channel, so
each is scaled by the factor that makes the same counter read the known size of the
plain 1 GiB copy that the counter program runs first.

    python -m paper_2202_02847_amd.profiling traffic --fetch F.csv --write W.csv \\
        --kernel "k_lpt<double, double, 1, 10, 10, false, false>" --bytes-per-launch B --out X.json

writes the per-launch fetch/write bytes, the scale factors and a hash of the kernel
sources; bench.py reports the traffic only while that hash matches the current sources.

    python -m paper_2202_02847_amd.profiling last --trace T_kernel_trace.csv --kernel NAME --last 10

gives the mean duration of the last dispatches of a kernel in a kernel trace (the launches at
the device's steady clock).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["csrc/lpt_impl.hpp", "csrc/k_lpt.hip", "csrc/layout.hpp", "csrc/device_common.hpp",
                  "csrc/kernels.hpp", "csrc/k_lpt_f64_m2l.hip"]
COPY_BYTES = 1 << 30  # the reference copy: 2^27 doubles read and written


def kernel_source_hash(files=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def _read(path):
    with open(path) as fh:
        return list(csv.DictReader(fh))


def _counter(rows, name, pred):
    return [float(r["Counter_Value"]) for r in rows if r["Counter_Name"] == name and pred(r["Kernel_Name"])]


def traffic(fetch_csv, write_csv, kernel, bytes_per_launch=None):
    fr, wr = _read(fetch_csv), _read(write_csv)
    is_copy = lambda k: "copyBuffer" in k  # noqa: E731
    is_kern = lambda k: kernel in k  # noqa: E731
    cf = max(_counter(fr, "FETCH_SIZE", is_copy))
    cw = max(_counter(wr, "WRITE_SIZE", is_copy))
    f_scale = COPY_BYTES / (cf * 1024.0)
    w_scale = COPY_BYTES / (cw * 1024.0)
    kf = _counter(fr, "FETCH_SIZE", is_kern)
    kw = _counter(wr, "WRITE_SIZE", is_kern)
    if not kf or not kw:
        raise SystemExit(f"kernel {kernel!r} not found in the counter files")
    fetch = sum(kf) / len(kf) * 1024.0 * f_scale
    write = sum(kw) / len(kw) * 1024.0 * w_scale
    out = {"kernel": kernel, "fetch_bytes": fetch, "write_bytes": write, "traffic_bytes": fetch + write,
           "fetch_scale": f_scale, "write_scale": w_scale, "dispatches": len(kf),
           "source_hash": kernel_source_hash()}
    if bytes_per_launch:
        out["algorithmic_bytes"] = bytes_per_launch
        out["traffic_over_algorithmic"] = (fetch + write) / bytes_per_launch
    return out


def last_dispatches(trace_csv, kernel, last):
    """Mean, min and max duration (us) of the last `last` dispatches of a kernel in a
    rocprofv3 kernel-trace file: the launches after the device reached its steady clock (the
    first 10-30 ms of work after idle run at a lower clock)."""
    rows = [r for r in _read(trace_csv) if kernel in r["Kernel_Name"]]
    if not rows:
        raise SystemExit(f"kernel {kernel!r} not found in {trace_csv}")
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rows[-last:]]
    return {"kernel": kernel, "dispatches": len(rows), "last": len(d), "mean_us": sum(d) / len(d),
            "min_us": min(d), "max_us": max(d)}


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    lt = sub.add_parser("last")
    lt.add_argument("--trace", required=True)
    lt.add_argument("--kernel", required=True)
    lt.add_argument("--last", type=int, default=10)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--bytes-per-launch", type=float, default=None)
    t.add_argument("--out", required=True)
    sub.add_parser("hash")
    args = ap.parse_args()
    if args.cmd == "hash":
        print(kernel_source_hash())
        return
    if args.cmd == "last":
        print(json.dumps(last_dispatches(args.trace, args.kernel, args.last), indent=1))
        return
    res = traffic(args.fetch, args.write, args.kernel, args.bytes_per_launch)
    with open(args.out, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main()
