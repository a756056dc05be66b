"""Short text summaries of rocprofv3 output, and the HBM traffic of a kernel
from two counter passes.

    python paper_2512_20927_amd/profile_summary.py stats <kernel_stats.csv> [--top N]
    python paper_2512_20927_amd/profile_summary.py pmc <fetch.csv> <write.csv> --kernel NAME
        [--family NAME]

``pmc`` reads the counter_collection CSVs of one ``--pmc FETCH_SIZE`` and one
``--pmc WRITE_SIZE`` run of a command that first made a plain 1 GiB device
copy. FETCH_SIZE and WRITE_SIZE are in KiB per dispatch; the copy (1 GiB read,
1 GiB written) calibrates each counter into bytes. It prints the kernel's
per-launch traffic and the hash of the kernel's sources, which a reader of the
summary uses to tell whether the kernel has changed since the counters were
taken.
"""

from __future__ import annotations

import argparse
import csv
import hashlib
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# sources that make up each profiled kernel (the common headers included)
KERNEL_SOURCES = {
    "render_quantile": ["paper_2512_20927_amd/csrc/render_quantile.hip",
                        "paper_2512_20927_amd/csrc/render_common.h",
                        "paper_2512_20927_amd/csrc/common.h"],
}

COPY_BYTES = 1 << 30


def source_hash(family: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[family]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stats(path: str, top: int = 16) -> str:
    rows = list(csv.DictReader(open(path)))
    out = ["%-64s %6s %10s %10s %10s %6s" % ("kernel", "calls", "avg_us", "min_us", "max_us", "pct")]
    for r in rows[:top]:
        out.append("%-64s %6s %10.1f %10.1f %10.1f %6.1f" % (
            r["Name"][:64], r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    return "\n".join(out)


def _per_dispatch(path: str, counter: str):
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
    return [(r["Kernel_Name"], float(r["Counter_Value"])) for r in rows]


def _calibration(rows) -> float:
    copies = [v for name, v in rows if name.startswith("__amd_rocclr_copyBuffer")]
    if not copies:
        raise SystemExit("no __amd_rocclr_copyBuffer dispatch to calibrate against")
    return COPY_BYTES / (max(copies) * 1024.0)


def pmc(fetch_csv: str, write_csv: str, kernel: str, family: str) -> str:
    fr, wr = _per_dispatch(fetch_csv, "FETCH_SIZE"), _per_dispatch(write_csv, "WRITE_SIZE")
    fs, ws = _calibration(fr), _calibration(wr)
    fk = [v for name, v in fr if kernel in name]
    wk = [v for name, v in wr if kernel in name]
    if not fk or not wk:
        raise SystemExit("kernel %r not found in the counter files" % kernel)
    f_kib, w_kib = sum(fk) / len(fk), sum(wk) / len(wk)
    traffic = f_kib * 1024.0 * fs + w_kib * 1024.0 * ws
    return "\n".join([
        "kernel: %s" % kernel,
        "dispatches: fetch %d, write %d" % (len(fk), len(wk)),
        "FETCH_SIZE_KiB_per_dispatch: %.1f" % f_kib,
        "WRITE_SIZE_KiB_per_dispatch: %.1f" % w_kib,
        "fetch_bytes_per_counted_KiB: %.2f  (from the 1 GiB copy)" % (fs * 1024.0),
        "write_bytes_per_counted_KiB: %.2f  (from the 1 GiB copy)" % (ws * 1024.0),
        "traffic_bytes_per_launch: %d" % round(traffic),
        "source_sha256: %s" % source_hash(family),
    ])


def read_summary(path: str) -> dict:
    """key: value lines of a summary file (other lines ignored)."""
    out = {}
    if not os.path.exists(path):
        return out
    for line in open(path):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            out[k.strip()] = v.strip()
    return out


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("--top", type=int, default=16)
    b = sub.add_parser("pmc")
    b.add_argument("fetch_csv")
    b.add_argument("write_csv")
    b.add_argument("--kernel", required=True)
    b.add_argument("--family", default="render_quantile", choices=sorted(KERNEL_SOURCES))
    args = ap.parse_args()
    if args.cmd == "stats":
        print(stats(args.csv, args.top))
    else:
        print(pmc(args.fetch_csv, args.write_csv, args.kernel, args.family))


if __name__ == "__main__":
    main()
