"""Summaries of rocprofv3 output for the repository's profiles/ folder.

kernel-stats: condenses a `rocprofv3 --kernel-trace --stats --output-format
csv` run into a short text table (per-kernel calls and durations).

traffic: combines two counter runs (`--pmc FETCH_SIZE`, then `--pmc
WRITE_SIZE`, both `--output-format csv`) of a program that launches the FFT
kernel and a plain copy kernel of known size, calibrates each counter by the
copy kernel (bytes it must move / what the counter reads for it), and writes
the calibrated HBM bytes per FFT launch with a hash of the kernel sources
the counters were taken with (bench.py reports the traffic only while that
hash still matches).

    python -m paper_2203_09384_amd.profiling kernel-stats DIR OUT.txt --command "..."
    python -m paper_2203_09384_amd.profiling traffic FETCH_DIR WRITE_DIR OUT.json \\
        --kernel k_fft_c32 --copy-kernel k_stream_copy --copy-bytes 536870912 \\
        --algorithmic-bytes 1073741824 --command "..."

counters: any other counters of a kernel (one `--pmc` run per counter
group), median per dispatch and per unit of work.

    python -m paper_2203_09384_amd.profiling counters OUT.txt DIR1 DIR2 ... \\
        --kernel k_fft_half_2048 --units 32768 --unit-name transform --command "..."
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ["paper_2203_09384_amd/csrc/device_fft.hpp", "paper_2203_09384_amd/csrc/fft_c32.hip",
                  "paper_2203_09384_amd/csrc/index_maps.hpp", "paper_2203_09384_amd/csrc/launch.hpp"]


def kernel_hash(sources=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _one(pattern):
    hits = glob.glob(pattern, recursive=True)
    if not hits:
        raise FileNotFoundError(pattern)
    return sorted(hits)[0]


def kernel_stats(run_dir: str, out: str, command: str, top: int = 8, name_filter: str = ""):
    """Summary of a rocprofv3 --stats run: the `top` kernels by total time
    (0: all) whose names contain `name_filter`."""
    path = _one(os.path.join(run_dir, "**", "*kernel_stats.csv"))
    rows = [r for r in csv.DictReader(open(path)) if name_filter in r["Name"]]
    top = top or len(rows)
    lines = [f"# rocprofv3 kernel statistics", f"# command: {command}", "",
             f"{'calls':>7} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'total_ms':>10}  kernel"]
    for r in rows[:top]:
        lines.append(f"{int(r['Calls']):>7} {float(r['AverageNs']) / 1e3:>10.2f} {float(r['MinNs']) / 1e3:>10.2f} "
                     f"{float(r['MaxNs']) / 1e3:>10.2f} {float(r['TotalDurationNs']) / 1e6:>10.2f}  {r['Name']}")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    return rows


def _counter(run_dir, name, kernel_sub):
    path = _one(os.path.join(run_dir, "**", "*counter_collection.csv"))
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
            if r["Counter_Name"] == name and kernel_sub in r["Kernel_Name"]]
    if not vals:
        raise ValueError(f"no {name} values for kernels matching {kernel_sub!r} in {path}")
    return statistics.median(vals), len(vals)


def traffic(fetch_dir, write_dir, out, kernel, copy_kernel, copy_bytes, algorithmic_bytes, command,
            kernel_instance="", tune_table="builtin"):
    f_k, nf = _counter(fetch_dir, "FETCH_SIZE", kernel)
    w_k, nw = _counter(write_dir, "WRITE_SIZE", kernel)
    f_c, _ = _counter(fetch_dir, "FETCH_SIZE", copy_kernel)
    w_c, _ = _counter(write_dir, "WRITE_SIZE", copy_kernel)
    f_scale = copy_bytes / f_c      # bytes per counted unit, from the copy kernel
    w_scale = copy_bytes / w_c
    fetch_b, write_b = f_k * f_scale, w_k * w_scale
    rec = {
        "kernel": kernel, "kernel_instance": kernel_instance or kernel, "kernel_hash": kernel_hash(),
        "tune_table": tune_table,
        "fetch_size_counter_median": f_k, "write_size_counter_median": w_k,
        "dispatches_counted": {"FETCH_SIZE": nf, "WRITE_SIZE": nw},
        "copy_kernel": copy_kernel, "copy_bytes_each_way": copy_bytes,
        "copy_fetch_counter": f_c, "copy_write_counter": w_c,
        "fetch_bytes_per_count": f_scale, "write_bytes_per_count": w_scale,
        "fetch_bytes_per_launch": fetch_b, "write_bytes_per_launch": write_b,
        "bytes_per_launch": fetch_b + write_b,
        "algorithmic_bytes_per_launch": algorithmic_bytes,
        "traffic_over_algorithmic": (fetch_b + write_b) / algorithmic_bytes,
        "command": command,
    }
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    return rec


def counters(run_dirs, out, kernel, command, units=0.0, unit_name="unit"):
    """Summary of one or more `rocprofv3 --pmc ... --output-format csv` runs:
    for every counter, the median value per dispatch of the kernels whose
    names contain `kernel`, and per `unit_name` when `units` (units of work
    per dispatch) is given."""
    rows = {}
    for d in run_dirs:
        path = _one(os.path.join(d, "**", "*counter_collection.csv"))
        for r in csv.DictReader(open(path)):
            if kernel in r["Kernel_Name"]:
                rows.setdefault(r["Counter_Name"], {}).setdefault(r.get("Dispatch_Id", len(rows)), 0.0)
                rows[r["Counter_Name"]][r.get("Dispatch_Id", len(rows))] += float(r["Counter_Value"])
    lines = ["# rocprofv3 counters", f"# command: {command}", f"# kernels matching: {kernel}", "",
             f"{'counter':<28} {'dispatches':>10} {'median/dispatch':>16}" +
             (f" {'per ' + unit_name:>16}" if units else "")]
    res = {}
    for name in sorted(rows):
        vals = list(rows[name].values())
        med = statistics.median(vals)
        res[name] = med
        line = f"{name:<28} {len(vals):>10} {med:>16.4g}"
        if units:
            line += f" {med / units:>16.4g}"
        lines.append(line)
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("kernel-stats")
    a.add_argument("run_dir")
    a.add_argument("out")
    a.add_argument("--command", required=True)
    a.add_argument("--top", type=int, default=8, help="kernels to list by total time (0: all)")
    a.add_argument("--filter", default="", help="only kernels whose names contain this")
    b = sub.add_parser("traffic")
    b.add_argument("fetch_dir")
    b.add_argument("write_dir")
    b.add_argument("out")
    b.add_argument("--kernel", required=True)
    b.add_argument("--copy-kernel", required=True)
    b.add_argument("--copy-bytes", type=float, required=True)
    b.add_argument("--algorithmic-bytes", type=float, required=True)
    b.add_argument("--command", required=True)
    b.add_argument("--kernel-instance", default="",
                   help="the template instance the counters belong to (as bench.py names it)")
    b.add_argument("--tune-table", default="builtin", help="the variant table the run planned with")
    c = sub.add_parser("counters")
    c.add_argument("out")
    c.add_argument("run_dirs", nargs="+")
    c.add_argument("--kernel", required=True)
    c.add_argument("--command", required=True)
    c.add_argument("--units", type=float, default=0.0, help="units of work per dispatch (for per-unit values)")
    c.add_argument("--unit-name", default="unit")
    args = ap.parse_args(argv)
    if args.cmd == "counters":
        counters(args.run_dirs, args.out, args.kernel, args.command, args.units, args.unit_name)
    elif args.cmd == "kernel-stats":
        kernel_stats(args.run_dir, args.out, args.command, args.top, args.filter)
    else:
        print(json.dumps(traffic(args.fetch_dir, args.write_dir, args.out, args.kernel, args.copy_kernel,
                                 args.copy_bytes, args.algorithmic_bytes, args.command, args.kernel_instance,
                                 args.tune_table), indent=1))


if __name__ == "__main__":
    main()
