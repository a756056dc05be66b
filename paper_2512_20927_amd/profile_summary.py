"""Short text summaries of rocprofv3 output, and the HBM traffic of a kernel
from two counter passes.

    python paper_2512_20927_amd/profile_summary.py stats <kernel_stats.csv> [--top N]
    python paper_2512_20927_amd/profile_summary.py pmc <fetch.csv> <write.csv> --kernel NAME
        [--family NAME]
    python paper_2512_20927_amd/profile_summary.py counters <counters.csv> --kernel NAME

``counters`` prints the per-dispatch mean of every counter collected for the
kernel, and the derived MFMA and VALU figures where their counters are present.
The collected values are sums over all counter instances; GRBM_GUI_ACTIVE is
therefore the busy cycles of one XCD times 8, and the derived figures use
G = GRBM_GUI_ACTIVE / 8: MFMA busy % = SQ_VALU_MFMA_BUSY_CYCLES / (G x SIMDs),
VALU busy % = SQ_ACTIVE_INST_VALU x 4 / (G x SIMDs) (the counter is in quad
cycles), bf16 MFMA flops = SQ_INSTS_VALU_MFMA_MOPS_BF16 x 512.

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
                        "paper_2512_20927_amd/csrc/quantile_select.h",
                        "paper_2512_20927_amd/csrc/render_common.h",
                        "paper_2512_20927_amd/csrc/common.h"],
    "render_dense": ["paper_2512_20927_amd/csrc/render_dense.hip",
                     "paper_2512_20927_amd/csrc/dense_walk.h",
                     "paper_2512_20927_amd/csrc/quantile_select.h",
                     "paper_2512_20927_amd/csrc/render_common.h",
                     "paper_2512_20927_amd/csrc/common.h"],
    "dense_backward": ["paper_2512_20927_amd/csrc/render_backward.hip",
                       "paper_2512_20927_amd/csrc/dense_walk.h",
                       "paper_2512_20927_amd/csrc/wave_ops.h",
                       "paper_2512_20927_amd/csrc/render_common.h",
                       "paper_2512_20927_amd/csrc/common.h"],
    "quantile_backward": ["paper_2512_20927_amd/csrc/render_quantile_backward.hip",
                          "paper_2512_20927_amd/csrc/quantile_select.h",
                          "paper_2512_20927_amd/csrc/wave_ops.h",
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


N_SIMD = 256 * 4  # MI355X: 256 CUs of 4 SIMDs
N_XCD = 8


def counters(path: str, kernel: str) -> str:
    rows = [r for r in csv.DictReader(open(path)) if kernel in r["Kernel_Name"]]
    if not rows:
        raise SystemExit("kernel %r not found" % kernel)
    per = {}
    durs = {}
    for r in rows:
        per.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        durs[r["Dispatch_Id"]] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    mean = {k: sum(v) / len(v) for k, v in per.items()}
    out = ["kernel: %s" % kernel, "dispatches: %d" % len(durs),
           "mean_duration_ms_under_counters: %.4f" % (1e3 * sum(durs.values()) / len(durs))]
    for k in sorted(mean):
        out.append("%s_per_dispatch: %.1f" % (k, mean[k]))
    gui = mean.get("GRBM_GUI_ACTIVE")
    if gui:
        gui /= N_XCD
        if "SQ_VALU_MFMA_BUSY_CYCLES" in mean:
            out.append("mfma_busy_pct: %.1f" % (100.0 * mean["SQ_VALU_MFMA_BUSY_CYCLES"] / (gui * N_SIMD)))
        if "SQ_ACTIVE_INST_VALU" in mean:
            out.append("valu_busy_pct: %.1f" % (100.0 * 4.0 * mean["SQ_ACTIVE_INST_VALU"] / (gui * N_SIMD)))
    if "SQ_INSTS_VALU_MFMA_MOPS_BF16" in mean:
        flops = mean["SQ_INSTS_VALU_MFMA_MOPS_BF16"] * 512.0
        out.append("bf16_mfma_flops_per_dispatch: %.4g" % flops)
        if gui:
            secs = gui / 2.4e9
            out.append("bf16_mfma_tflops_over_busy_time: %.1f  (GRBM_GUI_ACTIVE / 8 at 2.4 GHz)"
                       % (flops / secs / 1e12))
    return "\n".join(out)


def read_summary(path: str, kernel: str | None = None) -> dict:
    """key: value lines of a summary file (other lines ignored). With
    `kernel`, only the block that starts with "kernel: <kernel>" (files that
    summarise several kernels)."""
    out = {}
    if not os.path.exists(path):
        return out
    inside = kernel is None
    for line in open(path):
        if kernel is not None and line.startswith("kernel:"):
            inside = line.split(":", 1)[1].strip() == kernel
        if inside and ":" in line and not line.startswith(" "):
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
    c = sub.add_parser("counters")
    c.add_argument("csv")
    c.add_argument("--kernel", required=True)
    args = ap.parse_args()
    if args.cmd == "stats":
        print(stats(args.csv, args.top))
    elif args.cmd == "pmc":
        print(pmc(args.fetch_csv, args.write_csv, args.kernel, args.family))
    else:
        print(counters(args.csv, args.kernel))


if __name__ == "__main__":
    main()
