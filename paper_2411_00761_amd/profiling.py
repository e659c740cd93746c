"""Summaries of rocprofv3 output for the roofline figures.

    python -m paper_2411_00761_amd.profiling stats <kernel_stats.csv> <out.md> <command...>
    python -m paper_2411_00761_amd.profiling traffic <fetch.csv> <write.csv> <kernel> \
        <copy_kernel_regex> <copy_bytes> <out.json> <command...>

`stats` turns a --kernel-trace --stats CSV into a short markdown table.
`traffic` turns two --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) into
bytes per launch of one kernel, each scaled by what the same counter reads for a
plain device copy of known size in the same run (factor = copy bytes / counter
bytes), and records the SHA-256 of the kernel sources so a stale figure is not
reused after the kernels change.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["csrc/kernels_core.hip", "csrc/kernels_codec.hip", "csrc/lcp_common.h",
                  "csrc/lcp_internal.h"]


def source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def short_name(name: str) -> str:
    m = re.search(r"(k_\w+)", name)
    if m:
        return m.group(1)
    m = re.search(r"(__amd_rocclr_\w+|at::native::\w+)", name)
    return m.group(1) if m else name[:40]


def stats_markdown(path: str, command: str, top: int = 25) -> str:
    rows = list(csv.DictReader(open(path)))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    out = ["| kernel | calls | avg us | min us | max us | total ms | % |", "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows[:top]:
        out.append("| %s | %s | %.1f | %.1f | %.1f | %.2f | %.1f |" % (
            short_name(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))
    head = ["Command:", "", "```", command, "```", "",
            "Total GPU kernel time %.2f ms over %d kernel names." % (total / 1e6, len(rows)), ""]
    return "\n".join(head + out) + "\n"


def per_dispatch(path: str, counter: str):
    """{kernel short name: [(dispatch id, value summed over dimensions)]}"""
    acc = defaultdict(lambda: defaultdict(float))
    names = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        d = int(r["Dispatch_Id"])
        acc[d][counter] += float(r["Counter_Value"])
        names[d] = r["Kernel_Name"]
    out = defaultdict(list)
    for d in sorted(acc):
        out[names[d]].append((d, acc[d][counter]))
    return out


def traffic(fetch_csv, write_csv, kernel, copy_regex, copy_bytes):
    res = {}
    for label, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        pd = per_dispatch(path, counter)
        kv = [v for n, vals in pd.items() if short_name(n) in (kernel, "k_" + kernel)
              for _, v in vals]
        cv = [v for n, vals in pd.items() if re.search(copy_regex, n) for _, v in vals]
        if not kv or not cv:
            raise SystemExit(f"missing dispatches for {kernel} or the copy kernel in {path}")
        copy_kib = max(cv)  # the 256 MiB copies (smaller copies in the run are ignored)
        factor = copy_bytes / (copy_kib * 1024.0)
        mean_kib = sum(kv) / len(kv)
        res[label] = {"counter": counter, "kernel_kib_per_dispatch": mean_kib, "dispatches": len(kv),
                      "copy_kib": copy_kib, "copy_bytes": copy_bytes, "factor": factor,
                      "bytes_per_launch": mean_kib * 1024.0 * factor}
    res["traffic_bytes_per_launch"] = res["fetch"]["bytes_per_launch"] + res["write"]["bytes_per_launch"]
    res["kernel"] = kernel
    res["source_sha256"] = source_hash()
    return res


def main(argv):
    if argv[0] == "stats":
        md = stats_markdown(argv[1], " ".join(argv[3:]))
        open(argv[2], "w").write(md)
        print(md)
    elif argv[0] == "traffic":
        t = traffic(argv[1], argv[2], argv[3], argv[4], float(argv[5]))
        t["command"] = " ".join(argv[7:])
        open(argv[6], "w").write(json.dumps(t, indent=1) + "\n")
        print(json.dumps(t, indent=1))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
