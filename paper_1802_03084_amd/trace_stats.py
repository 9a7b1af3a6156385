"""Per-search kernel statistics from a rocprofv3 kernel trace.

A fused segment search launches one dedispersion pass (k_drs) per DM trial,
so the searches of a traced run can be told apart by counting k_drs launches.
For each search this prints its span and the mean duration of each kernel,
from the profiler's own timestamps (nothing is added to the schedule: the
figures hold for searches that ran without events, e.g. the timed steps of
bench.py).

    python -m paper_1802_03084_amd.trace_stats run_kernel_trace.csv NDM
"""
import collections
import csv
import re
import sys


def searches(path, ndm):
    """[(span_ms, {kernel: (mean_us, launches)})] per search, in time order."""
    iv = []
    with open(path) as f:
        for r in csv.DictReader(f):
            m = re.search(r"(k_\w+)", r.get("Kernel_Name", ""))
            if m:
                iv.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), m.group(1)))
    iv.sort()
    drs = [s for s, _, k in iv if k == "k_drs"]
    n = len(drs) // ndm
    bounds = [drs[i * ndm] for i in range(n)] + [float("inf")]
    out = []
    for i in range(n):
        sel = [x for x in iv if bounds[i] <= x[0] < bounds[i + 1]]
        acc = collections.defaultdict(list)
        for s, e, k in sel:
            acc[k].append((e - s) / 1e3)
        span = (max(e for _, e, _ in sel) - min(s for s, _, _ in sel)) / 1e6
        out.append((span, {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}))
    return out


def main(argv):
    if len(argv) != 3:
        print(__doc__.strip().splitlines()[-1].strip(), file=sys.stderr)
        return 2
    for i, (span, ks) in enumerate(searches(argv[1], int(argv[2]))):
        print(f"search {i + 1}: span {span:.1f} ms; " + ", ".join(
            f"{k} {m:.2f} us x{c}" for k, (m, c) in sorted(ks.items()) if k != "k_zero_i32"))
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
