"""Summaries of rocprofv3 output for the library's kernels.

    python -m paper_2412_17510_amd.profiling stats  <kernel_stats.csv> [--match NAME]
    python -m paper_2412_17510_amd.profiling trace  <kernel_trace.csv> [--match NAME]
    python -m paper_2412_17510_amd.profiling traffic --fetch F.csv --write W.csv \
            --copy-fetch CF.csv --copy-write CW.csv --copy-bytes B --match NAME --out T.json

`traffic` turns the per-dispatch L2-to-memory request counters of the named kernels
into bytes per launch, each request counted at its own size:
    read  = 32 TCC_EA0_RDREQ_32B + 64 TCC_EA0_RDREQ_64B + 128 TCC_EA0_RDREQ_128B
    write = 32 (TCC_EA0_WRREQ - TCC_EA0_WRREQ_64B) + 64 TCC_EA0_WRREQ_64B
(one rocprofv3 --pmc run for the read counters, one for the write counters), and
checks them against a plain copy of known size, whose bytes moved divided by the
counted bytes give the scale factors applied (about 1: the request sizes account
for the copy's traffic exactly).  The derived FETCH_SIZE counter of this device
counts a 128-byte request as 64 bytes, which is why it is not used.  The record
carries the hash of the kernel sources so that a benchmark can tell whether the
figure still describes the code.
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


READ_COUNTERS = ("TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_128B_sum", "TCC_EA0_RDREQ_sum")
WRITE_COUNTERS = ("TCC_EA0_WRREQ_sum", "TCC_EA0_WRREQ_64B_sum", "TCC_EA0_RDREQ_DRAM_sum")


def request_bytes(read_csv, write_csv, match):
    """Mean bytes per dispatch read and written by kernels whose name contains `match`,
    from the request-size-resolved counters; also the requests of no resolved size."""
    mean = lambda v: sum(v) / len(v)  # noqa: E731
    c = {}
    for path, names in ((read_csv, READ_COUNTERS), (write_csv, WRITE_COUNTERS)):
        for name in names:
            v = counter_values(path, name, match)
            if not v:
                raise SystemExit("traffic: no %s rows for kernel %r in %s" % (name, match, path))
            c[name] = mean(v)
    n32, n64, n128, nall = (c[k] for k in READ_COUNTERS)
    wr, wr64 = c["TCC_EA0_WRREQ_sum"], c["TCC_EA0_WRREQ_64B_sum"]
    return {"read_bytes": 32 * n32 + 64 * n64 + 128 * n128, "write_bytes": 32 * (wr - wr64) + 64 * wr64,
            "read_requests": {"32B": n32, "64B": n64, "128B": n128, "all": nall,
                              "unresolved": nall - (n32 + n64 + n128)},
            "write_requests": {"all": wr, "64B": wr64}, "dram_read_requests": c["TCC_EA0_RDREQ_DRAM_sum"],
            "launches": len(counter_values(read_csv, READ_COUNTERS[0], match))}


def traffic(read_csv, write_csv, copy_read_csv, copy_write_csv, copy_bytes, match, copy_match):
    """Bytes per library call (the named kernels' per-dispatch means added: one call may
    launch several kernels), scaled by the copy's bytes moved per counted byte."""
    cp = request_bytes(copy_read_csv, copy_write_csv, copy_match)
    kr = copy_bytes / cp["read_bytes"]
    kw = copy_bytes / cp["write_bytes"]
    per = {}
    rb = wb = 0.0
    for m in match.split("|"):
        r = request_bytes(read_csv, write_csv, m)
        per[m] = r
        rb += r["read_bytes"]
        wb += r["write_bytes"]
    return {"kernels": per, "copy": cp, "copy_bytes": copy_bytes, "read_scale": kr, "write_scale": kw,
            "read_bytes": rb * kr, "write_bytes": wb * kw, "traffic_bytes": rb * kr + wb * kw,
            "counters": {"read": list(READ_COUNTERS), "write": list(WRITE_COUNTERS)},
            "source_hash": source_hash()}


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
