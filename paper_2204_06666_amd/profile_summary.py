"""Summarise rocprofv3 output of the EHYB kernels into short text files.

Reads, from directories written by rocprofv3 (CSV output):
  * a --kernel-trace --stats run of bench.py  -> per-kernel statistics and
    the average of the EHYB dispatches inside the benchmark's timed window;
  * a --pmc FETCH_SIZE run and a --pmc WRITE_SIZE run of profile_kernels.py
    -> HBM bytes per EHYB launch, each counter scaled by what it reports for
    a copy of a known number of bytes.

Writes a markdown summary and a JSON file with the per-launch traffic and the
hash of the kernel source it was measured on.

    python3 paper_2204_06666_amd/profile_summary.py --trace DIR --fetch DIR --write DIR \
        --fetch-log FILE --out profiles/NAME.md --traffic profiles/NAME_traffic.json
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import re
import statistics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# FP64 values (dtype 0), one lane per row, plain loads (--kernel overrides)
KERNEL = "ehyb_spmv_kernel<0, 1, false>"


def _one(pattern):
    hits = sorted(glob.glob(pattern, recursive=True))
    if not hits:
        raise FileNotFoundError(pattern)
    return hits[0]


def kernel_source_hash():
    p = os.path.join(ROOT, "paper_2204_06666_amd", "csrc", "ehyb_device.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def trace_summary(trace_dir, warmup, steps, kernel=KERNEL, top=10):
    stats = list(csv.DictReader(open(_one(os.path.join(trace_dir, "**", "*kernel_stats.csv")))))
    rows = list(csv.DictReader(open(_one(os.path.join(trace_dir, "**", "*kernel_trace.csv")))))
    ehyb = sorted((r for r in rows if kernel in r["Kernel_Name"]), key=lambda r: int(r["Start_Timestamp"]))
    dur = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) for r in ehyb]
    window = dur[warmup:warmup + steps]
    return stats[:top], (statistics.mean(window) if window else None), len(ehyb)


def pmc_values(pmc_dir, counter, kernel=KERNEL):
    rows = list(csv.DictReader(open(_one(os.path.join(pmc_dir, "**", "*counter_collection.csv")))))
    out = {}
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        name = r["Kernel_Name"]
        key = "ehyb" if kernel in name else ("copy" if "probe_copy_kernel" in name else None)
        if key:
            out.setdefault(key, []).append(float(r["Counter_Value"]) * 1024.0)  # KiB -> bytes
    return {k: statistics.mean(v) for k, v in out.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--fetch-log", required=True, help="stdout of profile_kernels.py")
    ap.add_argument("--bench-json", default=None, help="bench.py output of the traced run")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--out", required=True)
    ap.add_argument("--traffic", required=True)
    ap.add_argument("--commands", default="", help="the commands that produced the inputs")
    ap.add_argument("--kernel", default=KERNEL, help="substring of the kernel name to summarise")
    ap.add_argument("--title", default="EHYB FP64 SpMV, 27-point stencil 100^3 (1e6 rows, 26,463,592 nnz)")
    ap.add_argument("--workload-name", default="stencil27-100^3")
    args = ap.parse_args()
    kernel = args.kernel

    stats, window_ns, n_disp = trace_summary(args.trace, args.warmup, args.steps, kernel)
    log = open(args.fetch_log).read()
    m = re.search(r"ehyb algorithmic_bytes=(\d+) copy_bytes_read=(\d+) copy_bytes_written=(\d+)", log)
    algo, copy_r, copy_w = (int(g) for g in m.groups())
    fetch = pmc_values(args.fetch, "FETCH_SIZE", kernel)
    write = pmc_values(args.write, "WRITE_SIZE", kernel)
    f_scale = copy_r / fetch["copy"]
    w_scale = copy_w / write["copy"]
    traffic = fetch["ehyb"] * f_scale + write["ehyb"] * w_scale
    kh = kernel_source_hash()
    bench = json.load(open(args.bench_json)) if args.bench_json else None

    lines = [f"# rocprofv3 summary: {args.title}", ""]
    if args.commands:
        lines += ["Commands (run from the repository root on one MI355X):", "", "```", args.commands.strip(),
                  "```", ""]
    lines += [f"Kernel source sha256[:16]: `{kh}`", "",
              "## Kernel statistics (--kernel-trace --stats)", "",
              "| kernel | calls | avg us | min us | max us |", "|---|---|---|---|---|"]
    for s in stats:
        name = s["Name"].replace("(anonymous namespace)::", "")
        name = (name[5:] if name.startswith("void ") else name).split("(")[0][:60] or "(unnamed)"
        lines.append(f"| `{name}` | {s['Calls']} | {float(s['AverageNs']) / 1e3:.2f} | "
                     f"{float(s['MinNs']) / 1e3:.2f} | {float(s['MaxNs']) / 1e3:.2f} |")
    lines += ["", f"Dispatches of `{kernel}` traced: {n_disp}. The benchmark's timed window is "
                  f"dispatches {args.warmup}..{args.warmup + args.steps - 1} (after {args.warmup} "
                  f"warm-up launches); their mean duration is **{window_ns / 1e3:.2f} us**."]
    if bench:
        lines.append(f"bench.py measured {bench['roofline']['launch_us']} us per launch with HIP "
                     f"events in the same run ({bench['value']} GFLOP/s).")
        lines.append("The kernel's overall average above also includes every other launch of the same "
                     "kernel symbol in that run.")
    lines += ["", "## HBM traffic per launch (--pmc FETCH_SIZE, then --pmc WRITE_SIZE)", "",
              f"Copy probe of {copy_r} bytes: FETCH_SIZE reads {fetch['copy']:.0f} bytes "
              f"(scale {f_scale:.4f}), WRITE_SIZE {write['copy']:.0f} bytes (scale {w_scale:.4f}).", "",
              f"| quantity | bytes |", "|---|---|",
              f"| FETCH_SIZE x scale | {fetch['ehyb'] * f_scale:.0f} |",
              f"| WRITE_SIZE x scale | {write['ehyb'] * w_scale:.0f} |",
              f"| traffic per launch | {traffic:.0f} |",
              f"| algorithmic bytes per launch | {algo} |",
              f"| traffic / algorithmic | {traffic / algo:.3f} |", ""]
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    open(args.out, "w").write("\n".join(lines) + "\n")
    json.dump({"kernel": kernel, "workload": args.workload_name, "kernel_source_sha256_16": kh,
               "bytes_per_launch": round(traffic), "fetch_bytes": round(fetch["ehyb"] * f_scale),
               "write_bytes": round(write["ehyb"] * w_scale), "fetch_scale": f_scale,
               "write_scale": w_scale, "algorithmic_bytes": algo,
               "timed_window_avg_us": round(window_ns / 1e3, 3)},
              open(args.traffic, "w"), indent=1)
    print(open(args.out).read())


if __name__ == "__main__":
    main()
