"""Summarise a rocprofv3 kernel trace (run_kernel_trace.csv): launches and
mean duration per kernel, and how many kernels ran at the same time.

Usage: python tests/trace_summary.py <run_kernel_trace.csv> [name filter]

Concurrency is taken over the launches whose name contains the filter
(default: the likelihood path's kernels, k_prep / k_mixed / k_thin64 /
k_finalize and their shared-launch variants): the largest number of them
running at once, and the share of the time at least one runs during which
two or more do.
"""
import csv
import sys
from collections import defaultdict


def main(path, filt=None):
    rows = list(csv.DictReader(open(path)))
    keys = ("k_prep", "k_mixed", "k_thin64", "k_finalize") if filt is None else (filt,)
    per = defaultdict(list)
    iv = []
    for r in rows:
        name = r["Kernel_Name"]
        t0, t1 = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        per[name].append(t1 - t0)
        if any(k in name for k in keys):
            iv.append((t0, t1, name))
    print(f"{'kernel':70s} {'launches':>8s} {'mean_us':>9s}")
    for name, d in sorted(per.items(), key=lambda kv: -len(kv[1])):
        print(f"{name[:70]:70s} {len(d):8d} {sum(d) / len(d) / 1e3:9.2f}")
    ev = sorted([(a, 1) for a, _, _ in iv] + [(b, -1) for _, b, _ in iv])
    cur = best = 0
    last = None
    busy = multi = 0
    for t, d in ev:
        if last is not None and cur > 0:
            busy += t - last
            if cur > 1:
                multi += t - last
        cur += d
        best = max(best, cur)
        last = t
    n_multi = sum(1 for _, _, n in iv if "_multi" in n)
    print(f"# likelihood-path launches: {len(iv)}, of them shared-launch kernels: {n_multi}")
    print(f"# at most {best} running at once; two or more during "
          f"{100.0 * multi / max(busy, 1):.1f}% of the time any runs")


if __name__ == "__main__":
    main(sys.argv[1], sys.argv[2] if len(sys.argv) > 2 else None)
