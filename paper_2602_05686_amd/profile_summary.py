"""Summarise a rocprofv3 --kernel-trace --output-format csv run as a short
markdown table: per kernel (and per launch grid for the streaming kernels),
calls, total and average duration."""

import collections
import csv
import sys


def short(name):
    name = name.replace("void ", "").replace("matamg::(anonymous namespace)::", "")
    return name.split("(")[0]


def main(trace_csv, top=30):
    rows = collections.defaultdict(lambda: [0, 0])
    with open(trace_csv) as f:
        for r in csv.DictReader(f):
            dur = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
            key = (short(r["Kernel_Name"]), int(r["Grid_Size_X"]) // int(r["Workgroup_Size_X"]))
            rows[key][0] += 1
            rows[key][1] += dur
    total = sum(v[1] for v in rows.values())
    print(f"total kernel time {total / 1e6:.1f} ms\n")
    print("| kernel | workgroups | calls | total ms | avg us |")
    print("|---|---:|---:|---:|---:|")
    for (k, g), (c, d) in sorted(rows.items(), key=lambda kv: -kv[1][1])[:top]:
        print(f"| `{k}` | {g} | {c} | {d / 1e6:.2f} | {d / c / 1e3:.1f} |")


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 30)
