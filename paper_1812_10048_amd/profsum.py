"""Short text summaries of rocprofv3 CSV output (kernel statistics and
per-dispatch hardware counters), for keeping next to the numbers they back.

    python -m paper_1812_10048_amd.profsum stats    DIR [--top N]
    python -m paper_1812_10048_amd.profsum counters DIR --copy-bytes B [--kernel NAME]

`stats` reads the `*_kernel_stats.csv` that `rocprofv3 --kernel-trace --stats
--output-format csv` writes and prints the busiest kernels.

`counters` reads `*_counter_collection.csv` from a `--pmc` run and prints, per
kernel, the number of dispatches and the mean and largest value of each
counter per dispatch.  `--copy-bytes B` names a plain device-to-device copy of
B bytes made during the run (the largest dispatch of the runtime's copy
kernel); FETCH_SIZE and WRITE_SIZE (KiB) of the kernel named by `--kernel` are
then scaled by B / (what the copy's own dispatch reads or writes), which turns
the counters into HBM bytes.  The digest of the sources that build that kernel
is printed with them: bench.py reports the traffic only while the digest still
matches.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))

# sources whose change invalidates measured traffic of the matrix-core kernel
TRAFFIC_SOURCES = ("csrc/assign_mfma.hip", "csrc/layout.hip", "csrc/dpmm_common.hpp")


def _code_only(text: str) -> str:
    """The source without its comments and with whitespace runs collapsed,
    so that an edit of a comment does not count as a change of the kernel."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def source_digest(files=TRAFFIC_SOURCES) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(HERE, f), encoding="utf-8") as fh:
            h.update(f.encode())
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def _find(root: str, suffix: str):
    files = sorted(glob.glob(os.path.join(root, "**", "*" + suffix), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {root}")
    return files


def _get(row, *names, default=""):
    for n in names:
        if n in row and row[n] != "":
            return row[n]
    return default


def short_name(k: str, width: int = 60) -> str:
    k = k.split("(")[0].strip()
    for pre in ("void ",):
        if k.startswith(pre):
            k = k[len(pre):]
    return k if len(k) <= width else k[:width - 3] + "..."


def stats(root: str, top: int) -> None:
    rows = []
    for f in _find(root, "kernel_stats.csv"):
        with open(f) as fh:
            rows.extend(csv.DictReader(fh))
    rows.sort(key=lambda r: -float(_get(r, "TotalDurationNs", default="0")))
    total = sum(float(_get(r, "TotalDurationNs", default="0")) for r in rows)
    print(f"{'kernel':60s} {'calls':>6s} {'avg us':>10s} {'min us':>10s} {'max us':>10s} {'total %':>8s}")
    for r in rows[:top]:
        tot = float(_get(r, "TotalDurationNs", default="0"))
        print(f"{short_name(_get(r, 'Name', 'KernelName')):60s} {int(float(_get(r, 'Calls', default='0'))):6d} "
              f"{float(_get(r, 'AverageNs', default='0')) / 1e3:10.2f} {float(_get(r, 'MinNs', default='0')) / 1e3:10.2f} "
              f"{float(_get(r, 'MaxNs', default='0')) / 1e3:10.2f} {100 * tot / max(total, 1):8.2f}")
    print(f"({len(rows)} kernels, {total / 1e6:.2f} ms of kernel time in all)")


def counters(root: str, copy_bytes: int, kernel: str | None) -> None:
    per = collections.defaultdict(lambda: collections.defaultdict(lambda: collections.defaultdict(float)))
    for f in _find(root, "counter_collection.csv"):
        with open(f) as fh:
            for row in csv.DictReader(fh):
                k = _get(row, "Kernel_Name", "Kernel-Name", default="?")
                c = _get(row, "Counter_Name", "Counter-Name", default="?")
                d = _get(row, "Dispatch_Id", "Dispatch-Id", "Correlation_Id", default="0")
                per[k][c][d] += float(_get(row, "Counter_Value", "Counter-Value", default="0"))
    def total(k):
        return sum(sum(v.values()) for v in per[k].values())
    print(f"{'kernel':60s} {'disp':>5s}  counter: mean / max per dispatch (KiB for *_SIZE)")
    ranked = sorted(per, key=lambda k: -total(k))
    shown = ranked[:25] + [k for k in ranked[25:] if "dpmm::" in k]   # every library kernel
    for k in shown:
        parts = []
        n = 0
        for c, dv in sorted(per[k].items()):
            n = max(n, len(dv))
            vals = list(dv.values())
            parts.append(f"{c}: {sum(vals) / len(vals):.6g} / {max(vals):.6g}")
        print(f"{short_name(k):60s} {n:5d}  " + "; ".join(parts))
    if not copy_bytes or not kernel:
        return
    copy = [k for k in per if "copyBuffer" in k]
    match = [k for k in per if kernel in k]
    if not copy or not match:
        print(f"no copy kernel or no kernel matching {kernel!r}")
        return
    print()
    print(f"calibration: plain copy of {copy_bytes} bytes (largest dispatch of {short_name(copy[0])})")
    for c in sorted(set(per[match[0]]) & set(per[copy[0]])):
        probe = max(per[copy[0]][c].values())
        if probe <= 0:
            continue
        factor = copy_bytes / (probe * 1024.0)
        vals = list(per[match[0]][c].values())
        mean = sum(vals) / len(vals)
        print(f"{c}: copy dispatch reads {probe:.6g} KiB -> {factor:.4f} bytes per counted byte")
        print(f"traffic {c} {short_name(match[0])}: {mean * 1024.0 * factor:.6e} bytes per dispatch "
              f"(raw {mean:.6g} KiB, {len(vals)} dispatches)")
    print(f"source digest: {source_digest()}")


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("dir")
    a.add_argument("--top", type=int, default=20)
    b = sub.add_parser("counters")
    b.add_argument("dir")
    b.add_argument("--copy-bytes", type=int, default=0)
    b.add_argument("--kernel", default=None)
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        stats(args.dir, args.top)
    else:
        counters(args.dir, args.copy_bytes, args.kernel)
    return 0


if __name__ == "__main__":
    sys.exit(main())
