"""Summaries of rocprofv3 CSV output for this library's kernels.

    python -m paper_0902_0699_amd.profsum stats DIR
        per-kernel table (calls, average / min / max duration) from the
        *kernel_stats.csv that `rocprofv3 --kernel-trace --stats --output-format csv`
        writes under DIR.

    python -m paper_0902_0699_amd.profsum traffic FETCH_DIR WRITE_DIR --kernel SUBSTR
            --copy SUBSTR --copy-bytes B [--skip N] [--take M] [--json OUT]
        HBM bytes per dispatch of the kernels whose name contains --kernel, from two
        `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs.  Each counter is
        scaled by what it reads for a plain copy kernel (name contains --copy) that
        reads B bytes and writes B bytes, so the figure does not depend on the
        counter's unit or on caching of the copy's traffic.  --skip / --take keep
        only dispatches N .. N+M-1 of the matching kernels in dispatch order (a run
        that launches one kernel for two workloads, one after the other).

    python -m paper_0902_0699_amd.profsum counters DIR --kernel SUBSTR [--skip N] [--take M]
        average per dispatch of every counter collected in DIR for those kernels.

    python -m paper_0902_0699_amd.profsum trace DIR --kernel SUBSTR [--min-ms T] [--skip N] [--take M]
        durations of one kernel's dispatches from the *kernel_trace.csv of a
        `--kernel-trace` run: those of at least T ms (a workload's size), then
        dispatches N .. N+M-1 of them in dispatch order.
"""

import argparse
import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def source_sha():
    """Hash of the kernel and plan sources (the same hash bench.py checks)."""
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def _one(pattern):
    files = sorted(glob.glob(pattern, recursive=True))
    if not files:
        raise SystemExit("no file matches %s" % pattern)
    return files


def kernel_stats(directory):
    rows = []
    for path in _one(os.path.join(directory, "**", "*kernel_stats.csv")):
        with open(path, newline="") as f:
            for r in csv.DictReader(f):
                rows.append({"name": r["Name"], "calls": int(r["Calls"]),
                             "total_ns": float(r["TotalDurationNs"]), "avg_ns": float(r["AverageNs"]),
                             "min_ns": float(r["MinNs"]), "max_ns": float(r["MaxNs"]),
                             "percent": float(r["Percentage"])})
    rows.sort(key=lambda r: -r["total_ns"])
    return rows


def counter_per_dispatch(directory, counter):
    """{kernel name: [value per dispatch]} for one counter (summed over dimensions),
    each list in dispatch order."""
    per = {}
    for path in _one(os.path.join(directory, "**", "*counter_collection.csv")):
        with open(path, newline="") as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                key = (r["Kernel_Name"], int(r["Dispatch_Id"]))
                per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    out = {}
    for (name, _), v in sorted(per.items(), key=lambda kv: kv[0][1]):
        out.setdefault(name, []).append(v)
    return out


def counter_names(directory):
    names = set()
    for path in _one(os.path.join(directory, "**", "*counter_collection.csv")):
        with open(path, newline="") as f:
            for r in csv.DictReader(f):
                names.add(r["Counter_Name"])
    return sorted(names)


def _match(d, sub, skip=0, take=None):
    hits = {k: v for k, v in d.items() if sub in k}
    if not hits:
        raise SystemExit("no kernel name contains %r; have: %s" % (sub, ", ".join(sorted(d))[:2000]))
    if len(hits) > 1 and (skip or take):
        raise SystemExit("--skip/--take need one kernel name; %r matches %s" % (sub, sorted(hits)))
    vals = [x for v in hits.values() for x in v]
    vals = vals[skip:] if take is None else vals[skip:skip + take]
    if not vals:
        raise SystemExit("no dispatch left after --skip/--take")
    return sum(vals) / len(vals), len(vals), sorted(hits)


def short(name, width=90):
    name = name.replace("(anonymous namespace)::", "").split("(")[0]
    return name if len(name) <= width else name[: width - 3] + "..."


def cmd_stats(args):
    rows = kernel_stats(args.dir)
    print("| kernel | calls | avg ms | min ms | max ms | % time |")
    print("|---|---|---|---|---|---|")
    for r in rows:
        print("| %s | %d | %.4f | %.4f | %.4f | %.1f |" % (short(r["name"]), r["calls"], r["avg_ns"] * 1e-6,
                                                          r["min_ns"] * 1e-6, r["max_ns"] * 1e-6, r["percent"]))


def cmd_traffic(args):
    res = {"kernel": args.kernel, "copy_kernel": args.copy, "copy_bytes_each_way": args.copy_bytes}
    if args.skip or args.take:
        res["dispatches"] = {"skip": args.skip, "take": args.take}
    for counter, d in (("FETCH_SIZE", args.fetch_dir), ("WRITE_SIZE", args.write_dir)):
        vals = counter_per_dispatch(d, counter)
        k_avg, k_n, k_names = _match(vals, args.kernel, args.skip, args.take)
        c_avg, c_n, _ = _match(vals, args.copy)
        scale = args.copy_bytes / c_avg
        res[counter] = {"kernel_raw_avg": k_avg, "kernel_dispatches": k_n, "copy_raw_avg": c_avg,
                        "copy_dispatches": c_n, "bytes_per_unit": scale, "kernel_bytes": k_avg * scale}
        res["kernel_names"] = [short(n, 200) for n in k_names]
    res["bytes_per_launch"] = res["FETCH_SIZE"]["kernel_bytes"] + res["WRITE_SIZE"]["kernel_bytes"]
    res["source_sha"] = source_sha()
    text = json.dumps(res, indent=1)
    if args.json:
        with open(args.json, "w") as f:
            f.write(text + "\n")
    print(text)


def cmd_counters(args):
    print("| counter | dispatches | average per dispatch |")
    print("|---|---|---|")
    for c in counter_names(args.dir):
        vals = counter_per_dispatch(args.dir, c)
        try:
            avg, n, _ = _match(vals, args.kernel, args.skip, args.take)
        except SystemExit:
            continue
        print("| %s | %d | %.6g |" % (c, n, avg))


def cmd_trace(args):
    ms = []
    for path in _one(os.path.join(args.dir, "**", "*kernel_trace.csv")):
        with open(path, newline="") as f:
            for r in csv.DictReader(f):
                if args.kernel not in r["Kernel_Name"]:
                    continue
                t = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6
                if t >= args.min_ms:
                    ms.append((int(r["Dispatch_Id"]), t, r["Kernel_Name"]))
    ms.sort()
    ms = ms[args.skip:] if args.take is None else ms[args.skip:args.skip + args.take]
    if not ms:
        raise SystemExit("no dispatch matches")
    names = sorted({short(n, 200) for _, _, n in ms})
    t = [x for _, x, _ in ms]
    print("| kernel | dispatches | avg ms | min ms | max ms |")
    print("|---|---|---|---|---|")
    print("| %s | %d | %.4f | %.4f | %.4f |" % (", ".join(names), len(t), sum(t) / len(t), min(t), max(t)))


def main(argv=None):
    ap = argparse.ArgumentParser(description="rocprofv3 CSV summaries")
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy", required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--json")
    t.add_argument("--skip", type=int, default=0)
    t.add_argument("--take", type=int, default=None)
    c = sub.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("--kernel", required=True)
    c.add_argument("--skip", type=int, default=0)
    c.add_argument("--take", type=int, default=None)
    r = sub.add_parser("trace")
    r.add_argument("dir")
    r.add_argument("--kernel", required=True)
    r.add_argument("--min-ms", type=float, default=0.0)
    r.add_argument("--skip", type=int, default=0)
    r.add_argument("--take", type=int, default=None)
    args = ap.parse_args(argv)
    {"stats": cmd_stats, "traffic": cmd_traffic, "counters": cmd_counters, "trace": cmd_trace}[args.cmd](args)


if __name__ == "__main__":
    main(sys.argv[1:])
