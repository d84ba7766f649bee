"""Turn rocprofv3 CSV output into the short text summaries kept beside the
benchmark: per-kernel durations (``--kernel-trace --stats``), HBM bytes per
dispatch from ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs scaled by a
copy kernel of known size, and per-dispatch counter averages.

    python -m paper_1401_8230_amd.rocprof_summary stats STATS_CSV --command CMD
    python -m paper_1401_8230_amd.rocprof_summary trace KERNEL_TRACE_CSV --command CMD \
        [--skip KERNEL_SUBSTR=N ...]
    python -m paper_1401_8230_amd.rocprof_summary traffic --fetch CSV --write CSV \\
        --kernel SUBSTR --copy-kernel SUBSTR --copy-bytes B --algorithmic-bytes A \\
        --command-fetch CMD --command-write CMD --json OUT.json --md OUT.md
    python -m paper_1401_8230_amd.rocprof_summary counters CSV --command CMD

Only the standard library is used; nothing here touches a GPU.
"""
import argparse
import csv
import json
import os
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_1401_8230_amd._build import kernel_source_hash  # noqa: E402


def short_name(name, width=90):
    return name if len(name) <= width else name[:width - 3] + "..."


def stats(path, command):
    rows = list(csv.DictReader(open(path)))
    lines = ["# rocprofv3 kernel statistics", "", "Command:", "", "```", command, "```", "",
             f"Kernel source sha256[:16]: `{kernel_source_hash()}`", "",
             "| kernel | calls | average us | min us | max us | % of GPU time |",
             "|---|---:|---:|---:|---:|---:|"]
    for r in rows:
        lines.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    return "\n".join(lines) + "\n"


def trace(path, command, skips):
    """Per-kernel dispatch durations from a --kernel-trace CSV: mean, median,
    min and max, after dropping the first N dispatches of the kernels named
    in `skips` ({substring: N}; the warm-up launches of a benchmark)."""
    durs = defaultdict(list)
    for r in csv.DictReader(open(path)):
        durs[r["Kernel_Name"]].append((int(r["Start_Timestamp"]),
                                       int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    lines = ["# rocprofv3 kernel trace, per-dispatch durations", "", "Command:", "", "```",
             command, "```", "", f"Kernel source sha256[:16]: `{kernel_source_hash()}`", ""]
    if skips:
        lines += ["Warm-up dispatches left out: " +
                  ", ".join(f"the first {n} of `{k}`" for k, n in skips.items()), ""]
    lines += ["| kernel | dispatches | mean us | median us | min us | max us |",
              "|---|---:|---:|---:|---:|---:|"]
    rows = []
    for name, v in durs.items():
        v = [d for _, d in sorted(v)]
        for sub, n in skips.items():
            if sub in name:
                v = v[n:]
        if not v:
            continue
        srt = sorted(v)
        rows.append((sum(v), name, len(v), sum(v) / len(v), srt[len(srt) // 2], srt[0], srt[-1]))
    for _, name, cnt, mean, med, lo, hi in sorted(rows, reverse=True):
        lines.append(f"| `{short_name(name)}` | {cnt} | {mean / 1e3:.1f} | {med / 1e3:.1f} | "
                     f"{lo / 1e3:.1f} | {hi / 1e3:.1f} |")
    return "\n".join(lines) + "\n"


def per_dispatch(path, counter):
    """{kernel name: [value per dispatch]} for one counter of a --pmc CSV."""
    acc = defaultdict(float)
    names = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        key = int(r["Dispatch_Id"])
        acc[key] += float(r["Counter_Value"])
        names[key] = r["Kernel_Name"]
    out = defaultdict(list)
    for key in sorted(acc):
        out[names[key]].append(acc[key])
    return out


def pick(table, substr):
    hits = [k for k in table if substr in k]
    if len(hits) != 1:
        raise SystemExit(f"kernel pattern {substr!r} matches {len(hits)} kernels: {hits}")
    return hits[0], table[hits[0]]


def traffic(a):
    result = {"kernel_sha256_16": kernel_source_hash(), "unit": "bytes per dispatch",
              "copy_bytes_each_way": a.copy_bytes, "algorithmic_bytes": a.algorithmic_bytes,
              "commands": {"FETCH_SIZE": a.command_fetch, "WRITE_SIZE": a.command_write}}
    md = ["# HBM traffic of the fill kernel (rocprofv3 counters)", "",
          "Counters are in KiB per dispatch.  Each is scaled by what the same counter",
          f"reads for a plain copy kernel that reads and writes {a.copy_bytes} bytes.", ""]
    total = 0.0
    for counter, path, cmd in (("FETCH_SIZE", a.fetch, a.command_fetch),
                               ("WRITE_SIZE", a.write, a.command_write)):
        table = per_dispatch(path, counter)
        kname, vals = pick(table, a.kernel)
        cname, cvals = pick(table, a.copy_kernel)
        copy_kib = sum(cvals) / len(cvals)
        factor = copy_kib * 1024.0 / a.copy_bytes
        kib = sum(vals) / len(vals)
        scaled = kib * 1024.0 / factor
        total += scaled
        result[counter] = {"kernel": kname, "dispatches": len(vals), "raw_kib_mean": kib,
                           "raw_kib_min": min(vals), "raw_kib_max": max(vals),
                           "copy_kernel": cname, "copy_raw_kib": copy_kib,
                           "calibration_factor": factor, "scaled_bytes": scaled}
        md += [f"## {counter}", "", "```", cmd, "```", "",
               f"- kernel `{short_name(kname)}`: {len(vals)} dispatches, mean {kib:.0f} KiB "
               f"(min {min(vals):.0f}, max {max(vals):.0f})",
               f"- copy kernel `{short_name(cname)}`: {copy_kib:.0f} KiB for {a.copy_bytes} "
               f"bytes, factor {factor:.4f}",
               f"- scaled: {scaled:.4e} bytes per dispatch", ""]
    result["bytes_per_launch"] = total
    md += ["## Total", "",
           f"- measured HBM bytes per dispatch: {total:.4e}",
           f"- algorithmic bytes per dispatch: {a.algorithmic_bytes:.4e} "
           f"(ratio {total / a.algorithmic_bytes:.4f})",
           f"- kernel source sha256[:16]: `{result['kernel_sha256_16']}`", ""]
    with open(a.json, "w") as f:
        json.dump(result, f, indent=1)
        f.write("\n")
    with open(a.md, "w") as f:
        f.write("\n".join(md))


def counters(path, command):
    acc = defaultdict(lambda: defaultdict(list))
    seen = defaultdict(float)
    for r in csv.DictReader(open(path)):
        seen[(r["Kernel_Name"], int(r["Dispatch_Id"]), r["Counter_Name"])] += float(r["Counter_Value"])
    for (k, _, c), v in seen.items():
        acc[k][c].append(v)
    names = sorted({c for k in acc for c in acc[k]})
    lines = ["# rocprofv3 counters, mean per dispatch", "", "Command:", "", "```", command, "```",
             "", f"Kernel source sha256[:16]: `{kernel_source_hash()}`", "",
             "| kernel | dispatches | " + " | ".join(names) + " |",
             "|---|---:|" + "---:|" * len(names)]
    for k in sorted(acc):
        n = max(len(v) for v in acc[k].values())
        cells = []
        for c in names:
            v = acc[k].get(c)
            cells.append(f"{sum(v) / len(v):.4g}" if v else "")
        lines.append(f"| `{short_name(k, 70)}` | {n} | " + " | ".join(cells) + " |")
    return "\n".join(lines) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--command", required=True)
    t = sub.add_parser("traffic")
    for name in ("fetch", "write", "kernel", "copy_kernel", "command_fetch", "command_write",
                 "json", "md"):
        t.add_argument("--" + name.replace("_", "-"), dest=name, required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--algorithmic-bytes", type=float, required=True)
    tr = sub.add_parser("trace")
    tr.add_argument("csv")
    tr.add_argument("--command", required=True)
    tr.add_argument("--skip", action="append", default=[],
                    help="KERNEL_SUBSTR=N: leave out the first N dispatches of that kernel")
    c = sub.add_parser("counters")
    c.add_argument("csv")
    c.add_argument("--command", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        sys.stdout.write(stats(a.csv, a.command))
    elif a.cmd == "trace":
        skips = {}
        for item in a.skip:
            k, n = item.rsplit("=", 1)
            skips[k] = int(n)
        sys.stdout.write(trace(a.csv, a.command, skips))
    elif a.cmd == "traffic":
        traffic(a)
    else:
        sys.stdout.write(counters(a.csv, a.command))


if __name__ == "__main__":
    main()
