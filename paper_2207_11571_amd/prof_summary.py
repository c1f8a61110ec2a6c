"""Summarise rocprofv3 output into the short text tables kept under profiles/.

    python -m paper_2207_11571_amd.prof_summary trace <dir> "<command>" > profiles/<name>.md
    python -m paper_2207_11571_amd.prof_summary counters <dir> <kernel-substring> <copy-bytes> "<command>"
    python -m paper_2207_11571_amd.prof_summary sq <dir1,dir2,...> "<kernel1;kernel2;...>" "<command>"
    python -m paper_2207_11571_amd.prof_summary hbm <fetch-dir> <write-dir> <kernel-substring> <copy-bytes> \
        <algorithmic-bytes> <mean-launch-us> "<command>" > profiles/<kernel>_counters.md

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


def _counter_mean(d, kernel, cname):
    """(mean value per dispatch of the kernel, largest value of a copy
    dispatch) for one counter of a --pmc run."""
    vals, copies = [], []
    for name, _, pmc in _dispatches(d):
        for c, v in pmc.items():
            if c != cname and not c.startswith(cname):
                continue
            if kernel in name:
                vals.append(v)
            if "copyBuffer" in name or "copy" in name.lower():
                copies.append(v)
    if not vals or not copies:
        raise SystemExit(f"no {cname} values for {kernel} in {d}")
    return sum(vals) / len(vals), max(copies), len(vals)


def hbm(fetch_dir, write_dir, kernel, copy_bytes, alg_bytes, mean_us, command):
    """HBM bytes per dispatch of one kernel from a FETCH_SIZE run and a
    WRITE_SIZE run (KiB per dispatch), each scaled by what the same counter
    reads for a device copy of copy_bytes, with the sha256 of the kernel
    source (bench.py uses the figure only while the source is unchanged)."""
    import hashlib
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = open(os.path.join(root, "paper_2207_11571_amd", "csrc", "dg_kernels.hip"), "rb").read()
    sha = hashlib.sha256(src).hexdigest()[:16]
    f_k, f_c, n_f = _counter_mean(fetch_dir, kernel, "FETCH_SIZE")
    w_k, w_c, n_w = _counter_mean(write_dir, kernel, "WRITE_SIZE")
    ff, fw = copy_bytes / (f_c * 1024.0), copy_bytes / (w_c * 1024.0)
    fb, wb = f_k * 1024.0 * ff, w_k * 1024.0 * fw
    tot = fb + wb
    print(f"# HBM traffic of `{kernel}`\n")
    print("Two counter runs (FETCH_SIZE, then WRITE_SIZE), each over the same command:\n")
    print(f"    {command}\n")
    print(f"Calibration: a device copy of {copy_bytes} bytes reads {f_c:.0f} KiB of FETCH_SIZE (factor {ff:.3f}) "
          f"and {w_c:.0f} KiB of WRITE_SIZE (factor {fw:.3f}).\n")
    print("| counter | dispatches | mean KiB / dispatch | factor | bytes / dispatch |")
    print("|---|---|---|---|---|")
    print(f"| FETCH_SIZE | {n_f} | {f_k:.1f} | {ff:.3f} | {fb:.0f} |")
    print(f"| WRITE_SIZE | {n_w} | {w_k:.1f} | {fw:.3f} | {wb:.0f} |\n")
    print(f"- hbm_bytes_per_launch: {tot:.0f}")
    print(f"- algorithmic_bytes_per_launch: {alg_bytes:.0f}")
    print(f"- traffic_over_algorithmic: {tot / alg_bytes:.3f}")
    print(f"- mean_launch_us: {mean_us:.2f}")
    print(f"- counter_TBs: {tot / (mean_us * 1e-6) / 1e12:.3f}")
    print("- source: paper_2207_11571_amd/csrc/dg_kernels.hip")
    print(f"- source_sha256_16: {sha}")


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
    elif sys.argv[1] == "hbm":
        hbm(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]), float(sys.argv[6]), float(sys.argv[7]),
            sys.argv[8])
    else:
        raise SystemExit(__doc__)
