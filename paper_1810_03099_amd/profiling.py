"""Summaries of rocprofv3 output for the committed profiles.

Two commands, both reading rocprofv3's CSV output (``--output-format csv``):

``python -m paper_1810_03099_amd.profiling stats STATS_CSV --title T --command C``
    prints a Markdown table of a ``--kernel-trace --stats`` run
    (``*_kernel_stats.csv``): calls, total / average duration and share per
    kernel.

``python -m paper_1810_03099_amd.profiling traffic --key K --kernel SUBSTR --source REL
      --fetch CSV --write CSV --copy-fetch CSV --copy-write CSV --copy-bytes B --command C``
    scales the kernel's ``FETCH_SIZE`` / ``WRITE_SIZE`` counters (KiB per
    dispatch, averaged over its dispatches) by what the same counters read for
    a device-to-device copy of B bytes each way, and records the resulting HBM
    bytes per launch under key K in ``profiles/traffic.json`` together with a
    digest of the kernel's source files (REL, or "a.hip+b.h" for several; a
    figure whose source digest no longer matches is stale and is not reported).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def source_digest(rel: str) -> str:
    """Digest of the kernel's source files ("a.hip+b.h": all of them, in order;
    one file gives the digest of that file alone)."""
    h = hashlib.sha256()
    for part in rel.split("+"):
        with open(os.path.join(ROOT, part), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short_name(n: str) -> str:
    n = n.replace("(anonymous namespace)::", "")
    m = re.match(r"(void )?([^(]+)\(", n)
    return m.group(2) if m else n


def stats_markdown(path: str, title: str, command: str) -> str:
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            rows.append((r["Name"], int(r["Calls"]), float(r["TotalDurationNs"]), float(r["AverageNs"]),
                         float(r["Percentage"])))
    rows.sort(key=lambda x: -x[2])
    out = [f"# {title}", "", "Command (run from the repository root on the GPU):", "", "```", command, "```", "",
           "rocprofv3 kernel statistics (durations in microseconds):", "",
           "| kernel | calls | total us | avg us | % |", "|---|---:|---:|---:|---:|"]
    for n, calls, tot, avg, pct in rows:
        out.append(f"| `{short_name(n)}` | {calls} | {tot / 1e3:.1f} | {avg / 1e3:.2f} | {pct:.1f} |")
    return "\n".join(out) + "\n"


def counter_mean(path: str, counter: str, match) -> tuple[float, int]:
    """Mean per dispatch of `counter` over the dispatches whose kernel name
    satisfies `match` (rocprofv3 counter_collection CSV)."""
    per = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter or not match(r["Kernel_Name"]):
                continue
            d = r.get("Dispatch_Id") or r.get("Correlation_Id") or str(len(per))
            per[d] = per.get(d, 0.0) + float(r["Counter_Value"])
    if not per:
        raise SystemExit(f"no {counter} rows for the kernel in {path}")
    return sum(per.values()) / len(per), len(per)


def is_copy(name: str) -> bool:
    """The calibration copy's kernel (a device-to-device copy), not the fill
    that initialises its source (a fill reads nothing, and averaged in it
    would understate the copy's FETCH_SIZE)."""
    n = name.lower()
    return "copy" in n and "fill" not in n


def traffic(a) -> dict:
    sub = a.kernel
    fk, nf = counter_mean(a.fetch, "FETCH_SIZE", lambda n: sub in n)
    wk, nw = counter_mean(a.write, "WRITE_SIZE", lambda n: sub in n)
    cf, _ = counter_mean(a.copy_fetch, "FETCH_SIZE", is_copy)
    cw, _ = counter_mean(a.copy_write, "WRITE_SIZE", is_copy)
    kib = a.copy_bytes / 1024.0
    sf, sw = kib / cf, kib / cw
    rec = {
        "source": a.source, "source_sha": source_digest(a.source), "kernel": sub,
        "fetch_kib_per_dispatch": fk, "write_kib_per_dispatch": wk, "dispatches": [nf, nw],
        "copy_bytes_each_way": a.copy_bytes, "copy_fetch_kib": cf, "copy_write_kib": cw,
        "fetch_scale": sf, "write_scale": sw,
        "bytes_per_launch": (fk * sf + wk * sw) * 1024.0,
        "fetch_bytes_per_launch": fk * sf * 1024.0, "write_bytes_per_launch": wk * sw * 1024.0,
        "command": a.command,
    }
    try:
        with open(TRAFFIC_FILE) as f:
            allrec = json.load(f)
    except (OSError, ValueError):
        allrec = {}
    allrec[a.key] = rec
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(allrec, f, indent=1, sort_keys=True)
        f.write("\n")
    return rec


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_1810_03099_amd.profiling")
    sp = ap.add_subparsers(dest="cmd", required=True)
    s = sp.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--title", required=True)
    s.add_argument("--command", required=True)
    t = sp.add_parser("traffic")
    for x in ("key", "kernel", "source", "fetch", "write", "copy_fetch", "copy_write", "command"):
        t.add_argument("--" + x.replace("_", "-"), dest=x, required=True)
    t.add_argument("--copy-bytes", dest="copy_bytes", type=int, required=True)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        sys.stdout.write(stats_markdown(a.csv, a.title, a.command))
    else:
        print(json.dumps(traffic(a), indent=1))


if __name__ == "__main__":
    main()
