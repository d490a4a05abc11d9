"""Turn rocprofv3 CSV output into the short text summaries kept in profiles/
and into the per-launch HBM traffic that bench.py reports.

  python -m paper_1910_13529_amd.profiling trace STATS_CSV --command CMD --out FILE.md
  python -m paper_1910_13529_amd.profiling traffic --fetch CSV --write CSV \
      --fetch-copy CSV --write-copy CSV --copy-mib N --solver custom --precision fp32 \
      --command-fetch CMD --command-write CMD --out profiles/traffic_counters.json [--by-name]

HBM traffic: FETCH_SIZE and WRITE_SIZE are read in KiB per dispatch, each in
its own rocprofv3 --pmc run, and scaled by what the same counter reads for a
plain device copy of known size (bytes moved / counter reading).  The
summary records the hash of the kernel sources it was taken with; bench.py
reports the traffic only while the sources are unchanged.
"""
import argparse
import collections
import csv
import hashlib
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")

CLASS_OF = (
    ("k_batch_curl_e", "batch_curl_e"), ("k_batch_curl_b", "batch_curl_b"), ("k_batch_push", "batch_push"),
    ("k_batch_jcorr", "batch_jcorr"), ("k_batch_add_j", "batch_add_j"), ("k_batch_merge", "batch_merge"),
    ("k_merge_boxes", "merge_boxes"), ("k_push_deposit", "push_deposit"), ("k_curl_e", "curl_e"), ("k_curl_b", "curl_b"),
    ("k_jcorr", "jcorr"), ("k_add_j", "add_j"), ("k_clear_j", "add_j"), ("k_new_slab", "window"), ("k_shift_fused", "window"), ("k_leap", "leap"),
    ("k_filter_rows", "filter"),
)


def kernel_source_hash():
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h", ".cpp")):
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode())
                h.update(f.read())
    return h.hexdigest()[:16]


def kernel_class(name):
    for key, cls in CLASS_OF:
        if key in name:
            return cls
    return None


def short_name(name):
    name = name.replace("(anonymous namespace)::", "")
    m = re.match(r"(?:void )?([\w:]+(?:<[^>]*>)?)", name)
    return m.group(1) if m else name[:60]


def counter_means(path, counter):
    """mean counter value per dispatch, keyed by kernel name"""
    agg = collections.defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in agg.items()}


def copy_scale(path, counter, copy_bytes):
    """bytes per counter unit, from the largest copy dispatch of the calibration run"""
    vals = counter_means(path, counter)
    kib = max(v for k, v in vals.items() if "copy" in k.lower())
    return copy_bytes / kib


def cmd_trace(args):
    rows = list(csv.DictReader(open(args.stats)))
    lines = ["# %s" % args.title, "", "Command:", "", "    %s" % args.command, "",
             "| kernel | calls | average (us) | total (ms) | share |", "|---|---|---|---|---|"]
    for r in rows[: args.top]:
        lines.append("| `%s` | %s | %.1f | %.3f | %.1f%% |" % (
            short_name(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3, float(r["TotalDurationNs"]) / 1e6,
            float(r["Percentage"])))
    if args.note:
        lines += ["", args.note]
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")


def cmd_traffic(args):
    copy_bytes = args.copy_mib << 20
    sf = copy_scale(args.fetch_copy, "FETCH_SIZE", copy_bytes)
    sw = copy_scale(args.write_copy, "WRITE_SIZE", copy_bytes)
    fetch = counter_means(args.fetch, "FETCH_SIZE")
    write = counter_means(args.write, "WRITE_SIZE")
    out = {"source_hash": kernel_source_hash(), "fetch_scale_bytes_per_unit": sf, "write_scale_bytes_per_unit": sw,
           "copy_calibration_bytes": copy_bytes, "command_fetch": args.command_fetch,
           "command_write": args.command_write, "kernels": {}}
    for name in fetch:
        cls = kernel_class(name)
        if cls is None or name not in write:
            continue
        # by name: one entry per kernel instantiation (e.g. the two species'
        # push launches of the beam-in-plasma run); else one per class
        key = short_name(name) if args.by_name else "%s/%s/%s" % (args.solver, args.precision, cls)
        if key in out["kernels"]:
            continue
        fb, wb = fetch[name] * sf, write[name] * sw
        out["kernels"][key] = {"kernel": short_name(name), "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                               "hbm_bytes_per_launch": fb + wb}
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("stats")
    t.add_argument("--command", required=True)
    t.add_argument("--title", default="rocprofv3 kernel trace")
    t.add_argument("--top", type=int, default=14)
    t.add_argument("--note", default="")
    t.add_argument("--out", required=True)
    c = sub.add_parser("traffic")
    for k in ("fetch", "write", "fetch_copy", "write_copy", "command_fetch", "command_write", "out"):
        c.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    c.add_argument("--copy-mib", type=int, required=True)
    c.add_argument("--solver", required=True)
    c.add_argument("--precision", required=True)
    c.add_argument("--by-name", action="store_true", help="key the kernels by their instantiated names")
    args = ap.parse_args()
    cmd_trace(args) if args.cmd == "trace" else cmd_traffic(args)


if __name__ == "__main__":
    main()
