"""Summarise a rocprofv3 --kernel-trace --output-format csv run as a short
markdown table: per kernel (and per launch grid for the streaming kernels),
calls, total and average duration.

With --levels, the V-cycles in the trace (each starts with the finest
level's first smoother step, k_smooth_first) are split by level instead:
a kernel belongs to the level whose vectors it writes, so a restriction
(k_stream mode 7, or mode 0 into the coarsest level) to the coarser level,
a prolongation (mode 2) to the finer one and the dense GEMV to the coarsest.
The table gives each level's launches and average time per V-cycle; a bench
log given with --log adds the level sizes it printed.

With --vcycle, the per-kernel table covers only the trace from the first
V-cycle on (a run that times V-cycles after one setup).

With --setup, only the last setup in the trace is summarised (from its
input validation, k_validate_csr, to the first V-cycle after it), per
kernel name, with the gaps between its kernels.

    python profile_summary.py <run_kernel_trace.csv> [top] [--vcycle]
    python profile_summary.py <run_kernel_trace.csv> --levels [--log bench.log]
    python profile_summary.py <run_kernel_trace.csv> --setup [top]
"""

import collections
import csv
import re
import sys


def short(name):
    name = name.replace("void ", "").replace("matamg::(anonymous namespace)::", "")
    return name.split("(")[0]


def load(trace_csv, starts=False):
    with open(trace_csv) as f:
        rows = list(csv.DictReader(f))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    out = [(short(r["Kernel_Name"]), int(r["Grid_Size_X"]) // int(r["Workgroup_Size_X"]),
            int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) for r in rows]
    if starts:
        return out, [(int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in rows]
    return out


def setup(trace_csv, top=25):
    seq, times = load(trace_csv, starts=True)
    val = [i for i, (k, _, _) in enumerate(seq) if k.startswith("k_validate_csr")]
    a = val[-1]
    b = next((i for i in range(a, len(seq)) if seq[i][0].startswith("k_smooth_first")), len(seq))
    win = seq[a:b]
    t = times[a:b]
    wall = t[-1][1] - t[0][0]
    busy = sum(d for _, _, d in win)
    # idle: time with no kernel running on any stream (kernels of the setup's
    # side stream overlap those of its main stream)
    gaps, end = 0, t[0][1]
    for st, en in t[1:]:
        gaps += max(0, st - end)
        end = max(end, en)
    print(f"setup window {wall / 1e6:.2f} ms: kernels {busy / 1e6:.2f} ms ({len(win)} launches, summed over "
          f"streams), no kernel running {gaps / 1e6:.2f} ms\n")
    per = collections.defaultdict(lambda: [0, 0])
    for k, _, d in win:
        name = k if k.startswith("k_stream") else k.split("<")[0]
        per[name][0] += 1
        per[name][1] += d
    print("| kernel | launches | total ms |")
    print("|---|---:|---:|")
    for k, (c, d) in sorted(per.items(), key=lambda kv: -kv[1][1])[:top]:
        print(f"| `{k}` | {c} | {d / 1e6:.2f} |")


def main(trace_csv, top=30, vcycle=False):
    rows = collections.defaultdict(lambda: [0, 0])
    seq = load(trace_csv)
    if vcycle:
        first = next((i for i, (k, _, _) in enumerate(seq) if k.startswith("k_smooth_first")), len(seq))
        seq = seq[first:]
    for k, g, dur in seq:
        rows[(k, g)][0] += 1
        rows[(k, g)][1] += dur
    total = sum(v[1] for v in rows.values())
    print(f"total kernel time {total / 1e6:.1f} ms\n")
    print("| kernel | workgroups | calls | total ms | avg us |")
    print("|---|---:|---:|---:|---:|")
    for (k, g), (c, d) in sorted(rows.items(), key=lambda kv: -kv[1][1])[:top]:
        print(f"| `{k}` | {g} | {c} | {d / 1e6:.2f} | {d / c / 1e3:.1f} |")


def stream_mode(k):
    m = re.match(r"k_stream<\w+, (\d+),", k)
    return int(m.group(1)) if m else None


def levels(trace_csv, log=None):
    seq = load(trace_csv)
    starts = [i for i, (k, _, _) in enumerate(seq) if k.startswith("k_smooth_first")]
    cycles = [seq[a:b] for a, b in zip(starts, starts[1:] + [len(seq)])]
    per = collections.defaultdict(lambda: [0, 0])  # level -> launches, ns (summed over cycles)
    walls = []
    for cyc in cycles:
        lev = 0
        for k, _, dur in cyc:
            mode = stream_mode(k)
            if mode in (7, 0):
                lev += 1
            elif mode == 2:
                lev -= 1
            per[lev][0] += 1
            per[lev][1] += dur
        walls.append(sum(d for _, _, d in cyc))
    sizes = {}
    if log:
        with open(log) as f:
            for line in f:
                m = re.search(r"level (\d+): n (\d+), nnz (\d+)", line)
                if m:
                    sizes[int(m.group(1))] = (int(m.group(2)), int(m.group(3)))
    nc = len(cycles)
    tot = sum(v[1] for v in per.values()) / nc
    print(f"{nc} V-cycles, kernel time {tot / 1e3:.1f} us per V-cycle\n")
    print("| level | rows | stored entries | launches per V-cycle | us per V-cycle | share |")
    print("|---:|---:|---:|---:|---:|---:|")
    for lv in sorted(per):
        c, d = per[lv]
        n, z = sizes.get(lv, ("", ""))
        print(f"| {lv} | {n} | {z} | {c / nc:.0f} | {d / nc / 1e3:.1f} | {100 * d / nc / tot:.1f}% |")


if __name__ == "__main__":
    a = sys.argv[1:]
    if "--setup" in a:
        rest = [x for x in a[1:] if x != "--setup"]
        setup(a[0], int(rest[0]) if rest else 25)
    elif "--levels" in a:
        lg = a[a.index("--log") + 1] if "--log" in a else None
        levels(a[0], lg)
    else:
        vc = "--vcycle" in a
        rest = [x for x in a[1:] if x != "--vcycle"]
        main(a[0], int(rest[0]) if rest else 30, vc)
