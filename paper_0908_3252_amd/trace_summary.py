"""Per-kernel duration table from a rocprofv3 kernel trace.

Reads ``<prefix>_kernel_trace.csv`` (``rocprofv3 --kernel-trace
--output-format csv``) and prints a markdown table with one row per kernel
name and launch shape (workgroups x, y, z and workgroup size): launches,
average / min / max duration in microseconds and share of the summed kernel
time, sorted by total time.

Usage: python -m paper_0908_3252_amd.trace_summary TRACE.csv [--top 30]
"""
from __future__ import annotations

import argparse
import collections
import csv
import re


def short_name(name: str) -> str:
    """Kernel name without return type and argument list, with the HIP
    vector types written as float2 / double2."""
    name = name.replace("HIP_vector_type<double, 2u>", "double2")
    name = name.replace("HIP_vector_type<float, 2u>", "float2")
    name = re.sub(r"^void ", "", name)
    depth, cut = 0, len(name)
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            cut = i
            break
    return name[:cut]


def _int(row, *names):
    for n in names:
        if n in row and row[n] != "":
            return int(float(row[n]))
    return 0


def summarize(path: str):
    groups = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3  # ns -> us
        wx, wy, wz = (_int(r, "Workgroup_Size_X", "Workgroup_Size"), _int(r, "Workgroup_Size_Y"),
                      _int(r, "Workgroup_Size_Z"))
        gx, gy, gz = (_int(r, "Grid_Size_X", "Grid_Size"), _int(r, "Grid_Size_Y"),
                      _int(r, "Grid_Size_Z"))
        wx, wy, wz = max(wx, 1), max(wy, 1), max(wz, 1)
        shape = f"{gx // wx}x{max(gy, 1) // wy}x{max(gz, 1) // wz}"
        groups[(short_name(r["Kernel_Name"]), shape, wx * wy * wz)].append(dur)
    total = sum(sum(v) for v in groups.values()) or 1.0
    rows = sorted(groups.items(), key=lambda kv: -sum(kv[1]))
    return rows, total


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("trace_csv")
    ap.add_argument("--top", type=int, default=30)
    args = ap.parse_args(argv)
    rows, total = summarize(args.trace_csv)
    print("| kernel | grid | wg | launches | avg us | min us | max us | share |")
    print("|---|---|---|---|---|---|---|---|")
    for (name, shape, wg), d in rows[: args.top]:
        print(f"| `{name}` | {shape} | {wg} | {len(d)} | {sum(d) / len(d):.2f} | {min(d):.2f} | "
              f"{max(d):.2f} | {100.0 * sum(d) / total:.1f}% |")


if __name__ == "__main__":
    main()
