"""Summarise rocprofv3 output into the short text tables kept under profiles/.

    python -m paper_2207_11571_amd.prof_summary trace <dir> "<command>" > profiles/<name>.md
    python -m paper_2207_11571_amd.prof_summary counters <dir> <kernel-substring> <copy-bytes> "<command>"
    python -m paper_2207_11571_amd.prof_summary sq <dir1,dir2,...> "<kernel1;kernel2;...>" "<command>"

`trace` reads the kernel dispatches of a --kernel-trace run (rocpd SQLite
database or kernel_stats/kernel_trace CSV) and prints per-kernel count, mean,
min, max and total duration.  `counters` reads a --pmc run (FETCH_SIZE or
WRITE_SIZE, KiB per dispatch), prints the per-dispatch values of the named
kernel and of the calibration copy (the largest __amd_rocclr_copyBuffer /
elementwise copy dispatch), and the scale factor copy-bytes / copy-reading.
"""
import csv
import glob
import os
import sqlite3
import sys
from collections import defaultdict


def _dispatches(d):
    """[(kernel_name, duration_ns, {counter: value})] from a rocprofv3 output dir."""
    out = []
    dbs = glob.glob(os.path.join(d, "**", "*.db"), recursive=True)
    if dbs:
        con = sqlite3.connect(dbs[0])
        cur = con.cursor()
        rows = cur.execute("select s.kernel_name, d.end - d.start, d.id from rocpd_kernel_dispatch d "
                           "join rocpd_info_kernel_symbol s on d.kernel_id = s.id order by d.start").fetchall()
        pmc = defaultdict(dict)
        try:
            for did, name, val in cur.execute(
                    "select e.event_id, i.name, e.value from rocpd_pmc_event e join rocpd_info_pmc i on e.pmc_id = i.id"):
                pmc[did][name] = pmc[did].get(name, 0.0) + val
        except sqlite3.Error:
            pass
        ev = {}
        try:
            for did, eid in cur.execute("select id, event_id from rocpd_kernel_dispatch"):
                ev[did] = eid
        except sqlite3.Error:
            pass
        for name, dur, did in rows:
            out.append((name, dur, pmc.get(ev.get(did), {})))
        return out
    for path in glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True):
        for r in csv.DictReader(open(path)):
            out.append((r["Kernel_Name"], int(r["End_Timestamp"]) - int(r["Start_Timestamp"]), {}))
    for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(path)):
            out.append((r["Kernel_Name"], 0, {r["Counter_Name"]: float(r["Counter_Value"])}))
    return out


def trace(d, command):
    stats = defaultdict(list)
    for name, dur, _ in _dispatches(d):
        stats[name.replace(".kd", "")].append(dur)
    rows = sorted(stats.items(), key=lambda kv: -sum(kv[1]))
    print("# rocprofv3 kernel trace summary\n")
    print(f"Command: `{command}`\n")
    print("| kernel | calls | mean us | min us | max us | total ms |")
    print("|---|---|---|---|---|---|")
    for name, ds in rows:
        print(f"| `{name[:90]}` | {len(ds)} | {sum(ds) / len(ds) / 1e3:.2f} | {min(ds) / 1e3:.2f} | "
              f"{max(ds) / 1e3:.2f} | {sum(ds) / 1e6:.3f} |")


def counters(d, kernel, copy_bytes, command):
    vals, copies = [], []
    for name, _, pmc in _dispatches(d):
        for cname, v in pmc.items():
            if kernel in name:
                vals.append((cname, v))
            if "copyBuffer" in name or "elementwise" in name or "copy" in name.lower():
                copies.append((cname, v))
    print(f"Command: `{command}`\n")
    if not vals or not copies:
        print("no counter values found")
        return
    cname = vals[0][0]
    mean_k = sum(v for _, v in vals) / len(vals)
    copy_read = max(v for _, v in copies)
    factor = float(copy_bytes) / (copy_read * 1024.0)
    print(f"- counter: {cname}")
    print(f"- kernel dispatches: {len(vals)}")
    print(f"- kernel mean KiB per dispatch: {mean_k:.1f}")
    print(f"- calibration copy KiB: {copy_read:.1f} for {copy_bytes} bytes")
    print(f"- scale factor: {factor:.4f}")
    print(f"- bytes per dispatch (scaled): {mean_k * 1024.0 * factor:.0f}")


def sq(dirs, kernels, command):
    """Mean per-dispatch SQ counters of the named kernels over several --pmc
    runs (one counter set each), also per wavefront (divided by SQ_WAVES)."""
    vals = defaultdict(lambda: defaultdict(list))
    for d in dirs:
        for name, _, pmc in _dispatches(d):
            for k in kernels:
                if k in name:
                    for c, v in pmc.items():
                        vals[k][c].append(v)
    print(f"Command (one run per counter set): `{command}`\n")
    for k in kernels:
        m = {c: sum(v) / len(v) for c, v in vals[k].items()}
        if not m:
            continue
        waves = m.get("SQ_WAVES", 0.0)
        print(f"### `{k}`\n")
        print("| counter | per dispatch | per wavefront |")
        print("|---|---|---|")
        for c in sorted(m):
            pw = f"{m[c] / waves:.1f}" if waves else ""
            print(f"| {c} | {m[c]:.0f} | {pw} |")
        print()


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(sys.argv[2], sys.argv[3])
    elif sys.argv[1] == "counters":
        counters(sys.argv[2], sys.argv[3], int(sys.argv[4]), sys.argv[5])
    elif sys.argv[1] == "sq":
        sq(sys.argv[2].split(","), sys.argv[3].split(";"), sys.argv[4])
    else:
        raise SystemExit(__doc__)
