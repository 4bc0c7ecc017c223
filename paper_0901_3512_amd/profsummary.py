"""Summarise rocprofv3 CSV output into short text reports.

  python -m paper_0901_3512_amd.profsummary stats  <dir-with-kernel_stats.csv> [--top N]
  python -m paper_0901_3512_amd.profsummary bytes  <fetch-dir> <write-dir> --kernel hop_kernel

`bytes` averages FETCH_SIZE and WRITE_SIZE (KiB per dispatch) over the dispatches of the named
kernel that follow the copy probe and scales each by what the same counter reads for a plain
device copy of exactly 1 GiB (the benchmark's --copy-probe, made just before its timed region: a
1 GiB copy reads and writes 1,048,576 KiB), giving HBM bytes per launch of the timed region.
"""
import argparse
import csv
import glob
import hashlib
import os

GIB_KIB = 1024.0 * 1024.0


def _one(pattern):
    files = sorted(glob.glob(pattern, recursive=True))
    if not files:
        raise SystemExit(f"no file matches {pattern}")
    return files[0]


def stats(d, top):
    path = _one(os.path.join(d, "**", "*kernel_stats.csv"))
    rows = list(csv.DictReader(open(path)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = [f"{'kernel':70s} {'calls':>7s} {'avg_us':>10s} {'total_ms':>10s} {'pct':>6s}"]
    for r in rows[:top]:
        name = r["Name"].replace("void ", "")[:70]
        out.append(f"{name:70s} {int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:10.2f} "
                   f"{float(r['TotalDurationNs']) / 1e6:10.2f} {100 * float(r['TotalDurationNs']) / tot:6.1f}")
    return "\n".join(out)


def _counter(d, name):
    path = _one(os.path.join(d, "**", "*counter_collection.csv"))
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == name]
    return rows


def _copy_reference(rows):
    """Counter value of the 1 GiB copy probe and the last dispatch id of the probe: the largest copy
    dispatches (the probe is by far the largest copy of a benchmark run)."""
    cp = [(float(r["Counter_Value"]), int(r["Dispatch_Id"])) for r in rows if "copyBuffer" in r["Kernel_Name"]]
    top = max(v for v, _ in cp)
    big = [(v, d) for v, d in cp if v >= 0.9 * top]
    return sum(v for v, _ in big) / len(big), max(d for _, d in big)


def bytes_per_launch(fetch_dir, write_dir, kernel):
    f = _counter(fetch_dir, "FETCH_SIZE")
    w = _counter(write_dir, "WRITE_SIZE")
    fref, fd = _copy_reference(f)
    wref, wd = _copy_reference(w)
    f_scale = GIB_KIB / fref
    w_scale = GIB_KIB / wref
    fk = [float(r["Counter_Value"]) for r in f if kernel in r["Kernel_Name"] and int(r["Dispatch_Id"]) > fd]
    wk = [float(r["Counter_Value"]) for r in w if kernel in r["Kernel_Name"] and int(r["Dispatch_Id"]) > wd]
    fetch = sum(fk) / len(fk) * f_scale * 1024.0
    write = sum(wk) / len(wk) * w_scale * 1024.0
    return dict(fetch_scale=f_scale, write_scale=w_scale, dispatches=len(fk), fetch_bytes=fetch,
                write_bytes=write, traffic_bytes=fetch + write)


def source_digest(path):
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("dir")
    a.add_argument("--top", type=int, default=20)
    b = sub.add_parser("bytes")
    b.add_argument("fetch_dir")
    b.add_argument("write_dir")
    b.add_argument("--kernel", default="hop_")
    b.add_argument("--source", default=os.path.join(os.path.dirname(__file__), "csrc", "dslash.hip"))
    args = ap.parse_args()
    if args.cmd == "stats":
        print(stats(args.dir, args.top))
    else:
        r = bytes_per_launch(args.fetch_dir, args.write_dir, args.kernel)
        print(f"kernel={args.kernel} dispatches={r['dispatches']}")
        print(f"fetch_scale={r['fetch_scale']:.4f} write_scale={r['write_scale']:.4f}")
        print(f"fetch_bytes_per_launch={r['fetch_bytes']:.6g}")
        print(f"write_bytes_per_launch={r['write_bytes']:.6g}")
        print(f"traffic_bytes_per_launch={r['traffic_bytes']:.6g}")
        print(f"source_sha256_16={source_digest(args.source)}")


if __name__ == "__main__":
    main()
