"""Summarise rocprofv3 output of bench.py runs into profiles/.

    python -m paper_1808_10375_amd.profsum --stats DIR/run_kernel_stats.csv \\
        --fetch DIR/run_counter_collection.csv --write DIR/run_counter_collection.csv \\
        --copy-fetch DIR/... --copy-write DIR/... --workload n2500_m5_f128_o1024x1024 \\
        --out profiles/views_2500x5_128.md --traffic profiles/traffic_views_2500x5_128.json \\
        --command "..."

FETCH_SIZE / WRITE_SIZE are KiB per dispatch.  Each is scaled by what the
same counter reads for an elementwise kernel that moves a known number of
bytes (bench.py --copy-calibration: reads and writes 1 GiB).
"""
from __future__ import annotations

import argparse
import collections
import csv
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

VIEW_KERNEL = "k_fourier_"  # the fused or streamed view kernel


def short(name: str) -> str:
    n = name.replace("void ", "")
    return n.split("(")[0]


def per_kernel(csv_path: str, counts=None):
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(csv_path)):
        agg[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    if counts is not None:
        counts.update({k: len(v) for k, v in agg.items()})
    return {k: sum(v) / len(v) for k, v in agg.items()}


def copy_factor(csv_path: str, true_bytes: int) -> float:
    """true bytes / counted bytes for the copy kernel (dispatches that moved
    data; the initial fill reads nothing)."""
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(csv_path))]
    vals = [v for v in vals if v > 0.25 * max(vals)]
    counted = sum(vals) / len(vals) * 1024.0
    return true_bytes / counted


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--stats", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--traffic")
    ap.add_argument("--command", default="")
    ap.add_argument("--title", default="")
    ap.add_argument("--view-kernels", default="",
                    help="comma-separated kernel-name parts whose traffic is summed as one "
                         "view update (the three-kernel path); default: the fused or "
                         "streamed view kernel")
    ap.add_argument("--mfma", help="counter CSV with SQ_VALU_MFMA_BUSY_CYCLES, "
                    "GRBM_GUI_ACTIVE and SQ_INSTS_VALU_MFMA_MOPS_BF16")
    ap.add_argument("--stalls", help="counter CSV with SQ_WAVE_CYCLES, SQ_WAIT_ANY, "
                    "SQ_WAIT_INST_ANY, SQ_ACTIVE_INST_VALU/LDS/VMEM, SQ_LDS_BANK_CONFLICT, "
                    "SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE")
    ap.add_argument("--simds", type=int, default=1024, help="SIMDs on the device")
    ap.add_argument("--xcds", type=int, default=8,
                    help="GRBM_GUI_ACTIVE instances summed in the CSV (one per XCD)")
    args = ap.parse_args()

    rows = list(csv.DictReader(open(args.stats)))
    lines = [f"# {args.title or 'rocprofv3 kernel statistics'}", "",
             f"Workload key: `{args.workload}`", ""]
    if args.command:
        lines += ["Commands (run from the repository root):", "", "```", args.command, "```",
                  ""]
    lines += ["| kernel | calls | avg us | min us | max us | % time |",
              "|---|---:|---:|---:|---:|---:|"]
    for r in rows:
        lines.append(f"| `{short(r['Name'])}` | {r['Calls']} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    traffic = None
    if args.fetch and args.write and args.copy_fetch and args.copy_write:
        ff = copy_factor(args.copy_fetch, args.copy_bytes)
        fw = copy_factor(args.copy_write, args.copy_bytes)
        counts = {}
        fetch = per_kernel(args.fetch, counts)
        write = per_kernel(args.write)
        lines += ["", f"HBM-side traffic per dispatch (FETCH_SIZE x {ff:.3f}, WRITE_SIZE x "
                  f"{fw:.3f}; factors from the 1 GiB copy calibration):", "",
                  "| kernel | read MB | written MB |", "|---|---:|---:|"]
        for k in fetch:
            if k in write and fetch[k] * 1024 * ff > 1e6:
                lines.append(f"| `{k}` | {fetch[k] * 1024 * ff / 1e6:.1f} | "
                             f"{write[k] * 1024 * fw / 1e6:.1f} |")
        # the view kernel with the most dispatches (the merged paths run a
        # second form, with the eps_psi partials, once per dm_iterate call)
        if args.view_kernels:
            parts = [p for p in args.view_kernels.split(",") if p]
            ks = [k for k in fetch if any(p + "<" in k or k.endswith(p) for p in parts)]
            vk = "views (3 kernels)" if ks else None
            if ks:
                traffic = {"read": sum(fetch[k] for k in ks) * 1024 * ff,
                           "written": sum(write[k] for k in ks) * 1024 * fw}
                traffic["total"] = traffic["read"] + traffic["written"]
                traffic["kernels"] = ks
        else:
            views = [k for k in fetch if VIEW_KERNEL in k]
            vk = max(views, key=lambda k: counts[k]) if views else None
            if vk:
                traffic = {"read": fetch[vk] * 1024 * ff, "written": write[vk] * 1024 * fw}
                traffic["total"] = traffic["read"] + traffic["written"]
    if args.mfma:
        per = collections.defaultdict(lambda: collections.defaultdict(list))
        for r in csv.DictReader(open(args.mfma)):
            per[short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
        lines += ["", "Matrix-core counters per dispatch (MFMA busy = "
                  "SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE per XCD x "
                  f"{args.simds} SIMDs); flops = SQ_INSTS_VALU_MFMA_MOPS_BF16 x 512):", "",
                  "| kernel | MFMA busy % | bf16 MFMA GFLOP | GPU cycles |",
                  "|---|---:|---:|---:|"]
        for k, d in per.items():
            m = {c: sum(v) / len(v) for c, v in d.items()}
            if m.get("SQ_INSTS_VALU_MFMA_MOPS_BF16", 0) <= 0:
                continue
            cyc = m["GRBM_GUI_ACTIVE"] / args.xcds
            util = 100.0 * m["SQ_VALU_MFMA_BUSY_CYCLES"] / (cyc * args.simds)
            lines.append(f"| `{k}` | {util:.1f} | "
                         f"{m['SQ_INSTS_VALU_MFMA_MOPS_BF16'] * 512 / 1e9:.1f} | {cyc:.3g} |")
    if args.stalls:
        per = collections.defaultdict(lambda: collections.defaultdict(list))
        for r in csv.DictReader(open(args.stalls)):
            per[short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
        lines += ["", "Where the waves' time goes, per dispatch (each SQ_* count over "
                  "SQ_WAVE_CYCLES, the summed lifetime of the kernel's waves; MFMA busy = "
                  "SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE per XCD x "
                  f"{args.simds} SIMDs)):", "",
                  "| kernel | waiting on memory/LDS (SQ_WAIT_ANY) | waiting to issue "
                  "(SQ_WAIT_INST_ANY) | issuing VALU | issuing LDS | LDS bank conflicts | "
                  "MFMA busy % |", "|---|---:|---:|---:|---:|---:|---:|"]
        for k, d in per.items():
            m = {c: sum(v) / len(v) for c, v in d.items()}
            wc = m.get("SQ_WAVE_CYCLES", 0)
            if wc < 1e8:
                continue
            mf = ""
            if m.get("SQ_VALU_MFMA_BUSY_CYCLES", 0) > 0 and m.get("GRBM_GUI_ACTIVE", 0) > 0:
                mf = f"{100 * m['SQ_VALU_MFMA_BUSY_CYCLES'] / (m['GRBM_GUI_ACTIVE'] / args.xcds * args.simds):.1f}"
            lines.append(f"| `{k}` | {m['SQ_WAIT_ANY'] / wc:.2f} | {m['SQ_WAIT_INST_ANY'] / wc:.2f} | "
                         f"{m['SQ_ACTIVE_INST_VALU'] / wc:.3f} | {m['SQ_ACTIVE_INST_LDS'] / wc:.3f} | "
                         f"{m['SQ_LDS_BANK_CONFLICT'] / wc:.3f} | {mf} |")
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    if args.traffic and traffic:
        import bench
        with open(args.traffic, "w") as fh:
            json.dump({"kernel_hash": bench.kernel_hash(), "workload": args.workload,
                       "kernel": vk, "bytes_per_launch": traffic["total"],
                       "read_bytes": traffic["read"], "written_bytes": traffic["written"]},
                      fh, indent=1)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
