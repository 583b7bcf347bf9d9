"""Summaries of rocprofv3 output for the library's kernels.

    python -m paper_2412_17510_amd.profiling stats  <kernel_stats.csv> [--match NAME]
    python -m paper_2412_17510_amd.profiling trace  <kernel_trace.csv> [--match NAME]
    python -m paper_2412_17510_amd.profiling traffic --fetch F.csv --write W.csv \
            --copy-fetch CF.csv --copy-write CW.csv --copy-bytes B --match NAME --out T.json

`traffic` turns the per-dispatch FETCH_SIZE / WRITE_SIZE counters (KiB) of the named
kernel into bytes per launch, scaled by what the same counters read for a plain copy
of known size (bytes moved / counter reading), and records the hash of the kernel
sources so that a benchmark can tell whether the figure still describes the code.
With --merge the output file holds a list of such records ({"records": [...]}), one per
launch configuration (the "plan" given in --extra): a record of the same plan is
replaced, and records taken from other kernel sources (another hash) are dropped.
"""
import argparse
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/spmv.hip", "csrc/mp_arith.hpp", "csrc/plan.cpp", "csrc/plan.hpp")


def source_hash(files=KERNEL_SOURCES):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _rows(path):
    with open(path) as f:
        return list(csv.DictReader(f))


def stats(path, match=None):
    out = []
    for r in _rows(path):
        if match and match not in r["Name"]:
            continue
        out.append((r["Name"], int(r["Calls"]), float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
                     float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    return out


def trace_durations(path, match):
    """Per-dispatch durations (us) and grid sizes of kernels whose name contains `match`."""
    out = []
    for r in _rows(path):
        if match in r["Kernel_Name"]:
            out.append(((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3, int(r["Grid_Size_X"])))
    return out


def counter_values(path, counter, match):
    vals = [float(r["Counter_Value"]) for r in _rows(path)
            if r["Counter_Name"] == counter and match in r["Kernel_Name"]]
    return vals


def traffic(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_bytes, match, copy_match):
    """Copy-calibrated bytes per launch; `match` may name several kernels ("a|b"), whose
    per-launch means are added (one library call launching several kernels)."""
    mean = lambda v: sum(v) / len(v)  # noqa: E731
    cf = counter_values(copy_fetch_csv, "FETCH_SIZE", copy_match)
    cw = counter_values(copy_write_csv, "WRITE_SIZE", copy_match)
    if not (cf and cw):
        raise SystemExit("traffic: no copy-kernel counter rows matching %r" % copy_match)
    # the copy reads and writes copy_bytes each: scale factors in bytes per KiB of reading
    kf = copy_bytes / mean(cf)
    kw = copy_bytes / mean(cw)
    per = {}
    fkib = wkib = 0.0
    for m in match.split("|"):
        f = counter_values(fetch_csv, "FETCH_SIZE", m)
        w = counter_values(write_csv, "WRITE_SIZE", m)
        if not (f and w):
            raise SystemExit("traffic: missing counter rows for kernel %r" % m)
        per[m] = {"fetch_kib": mean(f), "write_kib": mean(w), "launches": len(f)}
        fkib += mean(f)
        wkib += mean(w)
    fb = fkib * kf
    wb = wkib * kw
    return {"kernels": per, "fetch_kib_per_call": fkib, "write_kib_per_call": wkib,
            "copy_fetch_kib": mean(cf), "copy_write_kib": mean(cw), "copy_bytes": copy_bytes,
            "fetch_scale_bytes_per_kib": kf, "write_scale_bytes_per_kib": kw,
            "fetch_bytes": fb, "write_bytes": wb, "traffic_bytes": fb + wb, "source_hash": source_hash()}


def merge_record(path, rec):
    """Records of `path` (if any) with `rec` added: same-plan records replaced, records of
    other kernel sources dropped; ordered by plan."""
    old = []
    if os.path.exists(path):
        with open(path) as f:
            old = json.load(f).get("records", [])
    keep = [r for r in old if r.get("source_hash") == rec["source_hash"] and r.get("plan") != rec.get("plan")]
    keep.append(rec)
    return sorted(keep, key=lambda r: json.dumps(r.get("plan"), sort_keys=True))


def find_record(path, plan, n, hash_):
    """The record of `path` measured on these kernel sources, plan and matrix size, or None."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        recs = json.load(f).get("records", [])
    for r in recs:
        if r.get("source_hash") == hash_ and r.get("plan") == plan and r.get("n") == n:
            return r
    return None


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--match")
    t = sub.add_parser("trace")
    t.add_argument("csv")
    t.add_argument("--match", required=True)
    tr = sub.add_parser("traffic")
    for a in ("--fetch", "--write", "--copy-fetch", "--copy-write", "--match", "--out"):
        tr.add_argument(a, required=True)
    tr.add_argument("--copy-match", default="copy")
    tr.add_argument("--copy-bytes", type=float, required=True)
    tr.add_argument("--extra", default="{}", help="JSON object merged into the output (workload, plan)")
    tr.add_argument("--merge", action="store_true", help="keep one record per plan in a {records: [...]} file")
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        print("%-70s %6s %12s %12s %12s %7s" % ("kernel", "calls", "avg_us", "min_us", "max_us", "pct"))
        for name, calls, avg, mn, mx, pct in stats(args.csv, args.match):
            print("%-70s %6d %12.2f %12.2f %12.2f %7.2f" % (name[:70], calls, avg, mn, mx, pct))
    elif args.cmd == "trace":
        d = trace_durations(args.csv, args.match)
        ds = sorted(x[0] for x in d)
        print("dispatches %d  median %.2f us  min %.2f us  max %.2f us" % (len(d), ds[len(ds) // 2], ds[0], ds[-1]))
    else:
        res = traffic(args.fetch, args.write, args.copy_fetch, args.copy_write, args.copy_bytes, args.match,
                      args.copy_match)
        res.update(json.loads(args.extra))
        out = res
        if args.merge:
            out = {"records": merge_record(args.out, res)}
        with open(args.out, "w") as f:
            json.dump(out, f, indent=1)
        print(json.dumps(res, indent=1))
    return 0


if __name__ == "__main__":
    sys.exit(main())
