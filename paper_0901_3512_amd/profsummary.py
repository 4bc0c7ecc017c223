"""Summarise rocprofv3 CSV output into short text reports.

  python -m paper_0901_3512_amd.profsummary stats  <dir-with-kernel_stats.csv> [--top N]
  python -m paper_0901_3512_amd.profsummary bytes  <fetch-dir> <write-dir> --kernel hop_kernel
  python -m paper_0901_3512_amd.profsummary counters <dir-with-counter_collection.csv> --kernel proj_kernel
  python -m paper_0901_3512_amd.profsummary markers  <dir-with-marker_api_stats.csv>

`bytes` averages FETCH_SIZE and WRITE_SIZE (KiB per dispatch) over the dispatches of the named
kernel between the copy probe and the next 1 GiB copy, and scales each by what the same counter
reads for a plain device copy of exactly 1 GiB (the benchmark's --copy-probe, made just before its
timed region: a 1 GiB copy reads and writes 1,048,576 KiB), giving HBM bytes per launch of the
timed region.
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


def markers(d):
    """The roctx ranges of a --marker-trace run: calls, average and total milliseconds per name."""
    path = _one(os.path.join(d, "**", "*marker_api_stats.csv"))
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = [f"{'range':50s} {'calls':>7s} {'avg_ms':>10s} {'total_ms':>10s}"]
    for r in rows:
        out.append(f"{r['Name'][:50]:50s} {int(r['Calls']):7d} {float(r['AverageNs']) / 1e6:10.3f} "
                   f"{float(r['TotalDurationNs']) / 1e6:10.1f}")
    return "\n".join(out)


def _counter(d, name):
    path = _one(os.path.join(d, "**", "*counter_collection.csv"))
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == name]
    return rows


def _copy_window(rows):
    """The 1 GiB copy probe in a counter trace: (mean counter value of its copies, dispatch id of its
    last copy, dispatch id of the next copy of that size or None).  The probe is a run of two or more
    back-to-back copies (no other dispatch in between) whose values agree within 10%: the first such
    run within 10% of the largest one, since smaller runs (a batch placing its configurations, say)
    can come first and other large copies (a basis growing by device copies) are single.  Without such
    a run: the first run of copies within 10% of the largest.  A later copy of the probe's size (the
    benchmark's copy-rate measurement after its timed region) ends the window."""
    cp = sorted((int(r["Dispatch_Id"]), float(r["Counter_Value"])) for r in rows if "copyBuffer" in r["Kernel_Name"])
    ids = sorted({int(r["Dispatch_Id"]) for r in rows})

    def adjacent(a, b):
        return not any(a < x < b for x in ids)

    def close(u, v):
        return abs(u - v) <= 0.1 * max(u, v)

    runs = []
    k = 0
    while k < len(cp) - 1:
        if adjacent(cp[k][0], cp[k + 1][0]) and close(cp[k][1], cp[k + 1][1]):
            run = [cp[k], cp[k + 1]]
            for d, v in cp[k + 2:]:
                if not (adjacent(run[-1][0], d) and close(run[0][1], v)):
                    break
                run.append((d, v))
            runs.append(run)
            k += len(run)
        else:
            k += 1
    probe = None
    if runs:
        top = max(r[0][1] for r in runs)
        probe = next(r for r in runs if close(r[0][1], top))
    if probe is None:
        top = max(v for _, v in cp)
        big = [(d, v) for d, v in cp if v >= 0.9 * top]
        probe = [big[0]]
        for d, v in big[1:]:
            if not adjacent(probe[-1][0], d):
                break
            probe.append((d, v))
    ref = sum(v for _, v in probe) / len(probe)
    last = probe[-1][0]
    after = [d for d, v in cp if d > last and close(ref, v)]
    return ref, last, (after[0] if after else None)


def bytes_per_launch(fetch_dir, write_dir, kernel):
    f = _counter(fetch_dir, "FETCH_SIZE")
    w = _counter(write_dir, "WRITE_SIZE")
    fref, f0, f1 = _copy_window(f)
    wref, w0, w1 = _copy_window(w)
    f_scale = GIB_KIB / fref
    w_scale = GIB_KIB / wref

    def inside(r, a, b):
        d = int(r["Dispatch_Id"])
        return d > a and (b is None or d < b)

    fk = [float(r["Counter_Value"]) for r in f if kernel in r["Kernel_Name"] and inside(r, f0, f1)]
    wk = [float(r["Counter_Value"]) for r in w if kernel in r["Kernel_Name"] and inside(r, w0, w1)]
    if not fk or not wk:
        raise SystemExit(f"no {kernel} dispatch between the copy probe and the next 1 GiB copy")
    fetch = sum(fk) / len(fk) * f_scale * 1024.0
    write = sum(wk) / len(wk) * w_scale * 1024.0
    return dict(fetch_scale=f_scale, write_scale=w_scale, dispatches=len(fk), fetch_bytes=fetch,
                write_bytes=write, traffic_bytes=fetch + write)


def counters(d, kernel):
    """Per kernel name containing `kernel`: dispatches, summed dispatch time, every counter's total,
    and (when collected) the matrix-core busy fraction and MFMA TFLOP/s.  GRBM_GUI_ACTIVE is summed
    over the 8 XCDs, SQ_VALU_MFMA_BUSY_CYCLES over the 1024 SIMDs; a MOPS unit is 512 flops."""
    path = _one(os.path.join(d, "**", "*counter_collection.csv"))
    agg, dur = {}, {}
    for r in csv.DictReader(open(path)):
        if kernel not in r["Kernel_Name"]:
            continue
        name = r["Kernel_Name"].split("(")[0].replace("void ", "")
        agg.setdefault(name, {}).setdefault(r["Counter_Name"], 0.0)
        agg[name][r["Counter_Name"]] += float(r["Counter_Value"])
        dur.setdefault(name, {})[r["Dispatch_Id"]] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    out = []
    for name, c in agg.items():
        n = len(dur[name])
        t = sum(dur[name].values()) * 1e-9
        line = f"{name}: dispatches {n}, total {t * 1e3:.2f} ms"
        for key in sorted(c):
            line += f", {key} {c[key]:.4g}"
        if "GRBM_GUI_ACTIVE" in c and "SQ_VALU_MFMA_BUSY_CYCLES" in c:
            line += f", MFMA busy fraction {c['SQ_VALU_MFMA_BUSY_CYCLES'] / (c['GRBM_GUI_ACTIVE'] / 8 * 1024):.4f}"
        for p in ("F64", "F32"):
            m = c.get(f"SQ_INSTS_VALU_MFMA_MOPS_{p}")
            if m:
                line += f", {p} TFLOP/s {m * 512 / t / 1e12:.2f}"
        if "FETCH_SIZE" in c:
            line += f", fetch KiB/dispatch {c['FETCH_SIZE'] / n:.4g}"
        out.append(line)
    return "\n".join(out)


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
    mk = sub.add_parser("markers")
    mk.add_argument("dir")
    c = sub.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("--kernel", default="proj_kernel")
    args = ap.parse_args()
    if args.cmd == "stats":
        print(stats(args.dir, args.top))
    elif args.cmd == "markers":
        print(markers(args.dir))
    elif args.cmd == "counters":
        print(counters(args.dir, args.kernel))
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
