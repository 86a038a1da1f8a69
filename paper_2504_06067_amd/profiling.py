"""Helpers that turn rocprofv3 output into the short summaries kept with the
benchmark, and read the HBM traffic figure back.

  python -m paper_2504_06067_amd.profiling stats <kernel_stats.csv> <out.md> <title> <command>
  python -m paper_2504_06067_amd.profiling traffic <fetch_counter.csv> <write_counter.csv> \\
        <kernel substring> <copy kernel substring> <copy bytes> <out.json> <command...>

The traffic record scales each counter (FETCH_SIZE, WRITE_SIZE: KiB per
dispatch) by what the same counter reads for a plain device-to-device copy
of known size in the same run, and stores the SHA-256 of the kernel's source
file: once that source changes the figure no longer applies and
``read_traffic`` returns None.
"""
import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DOMINANCE_SOURCE = os.path.join(ROOT, "paper_2504_06067_amd", "csrc", "ndsort.hip")


def source_digest(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def kernel_stats_md(stats_csv, title, command):
    rows = list(csv.DictReader(open(stats_csv)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    out = [f"# {title}", "", "Command (from the repository root, one MI355X):", "", "```",
           command, "```", "",
           "| kernel | calls | avg us | min us | max us | share |",
           "|---|---:|---:|---:|---:|---:|"]
    for r in rows:
        name = r["Name"].split("(")[0].replace("void ", "")
        out.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                   f"{float(r['Percentage']):.1f}% |")
    out += ["", f"Sum of kernel time over the run: {tot / 1e6:.3f} ms.", ""]
    return "\n".join(out)


def counter_per_dispatch(counter_csv, counter):
    """{kernel name: [value per dispatch]} for one counter."""
    per = {}
    for r in csv.DictReader(open(counter_csv)):
        if r.get("Counter_Name") != counter:
            continue
        per.setdefault(r["Kernel_Name"], {}).setdefault(r["Dispatch_Id"], 0.0)
        per[r["Kernel_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"])
    return {k: list(v.values()) for k, v in per.items()}


def _mean_for(per, sub):
    vals = [v for k, vs in per.items() if sub in k for v in vs]
    if not vals:
        raise KeyError(f"no dispatch of a kernel matching {sub!r}")
    return sum(vals) / len(vals), len(vals)


def _max_for(per, sub):
    """The largest dispatch of a matching kernel (the calibration copy among
    the small copies a run also makes)."""
    vals = [v for k, vs in per.items() if sub in k for v in vs]
    if not vals:
        raise KeyError(f"no dispatch of a kernel matching {sub!r}")
    return max(vals)


def traffic_record(fetch_csv, write_csv, kernel_sub, copy_sub, copy_bytes, command):
    f = counter_per_dispatch(fetch_csv, "FETCH_SIZE")
    w = counter_per_dispatch(write_csv, "WRITE_SIZE")
    kf, nf = _mean_for(f, kernel_sub)
    kw, nw = _mean_for(w, kernel_sub)
    cf = _max_for(f, copy_sub)
    cw = _max_for(w, copy_sub)
    sf = copy_bytes / (cf * 1024.0)
    sw = copy_bytes / (cw * 1024.0)
    return {
        "kernel": kernel_sub,
        "source": os.path.relpath(DOMINANCE_SOURCE, ROOT),
        "source_sha256": source_digest(DOMINANCE_SOURCE),
        "fetch_kib_per_dispatch": kf, "write_kib_per_dispatch": kw,
        "dispatches": [nf, nw],
        "copy_kernel": copy_sub, "copy_bytes": copy_bytes,
        "copy_fetch_kib": cf, "copy_write_kib": cw,
        "scale_fetch": sf, "scale_write": sw,
        "fetch_bytes": kf * 1024.0 * sf, "write_bytes": kw * 1024.0 * sw,
        "traffic_bytes": kf * 1024.0 * sf + kw * 1024.0 * sw,
        "command": command,
    }


def read_traffic(path):
    """The traffic record at `path` if it still applies to the current
    source of its kernel, else None."""
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    src = os.path.join(ROOT, rec.get("source", ""))
    if not os.path.exists(src) or source_digest(src) != rec.get("source_sha256"):
        return None
    return rec


def main(argv):
    if argv[0] == "stats":
        stats_csv, out, title, command = argv[1:5]
        with open(out, "w") as f:
            f.write(kernel_stats_md(stats_csv, title, command))
    elif argv[0] == "traffic":
        fetch_csv, write_csv, ksub, csub, cbytes, out = argv[1:7]
        rec = traffic_record(fetch_csv, write_csv, ksub, csub, float(cbytes), " ".join(argv[7:]))
        with open(out, "w") as f:
            json.dump(rec, f, indent=1)
            f.write("\n")
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
