"""Summarise rocprofv3 output of the EHYB kernels into short text files.

Reads, from directories written by rocprofv3 (CSV output):
  * a --kernel-trace --stats run of bench.py  -> per-kernel statistics and
    the average of the EHYB dispatches inside the benchmark's timed window;
  * a --pmc FETCH_SIZE run and a --pmc WRITE_SIZE run of profile_kernels.py
    -> HBM bytes per EHYB launch, each counter scaled by what it reports for
    a copy of a known number of bytes;
  * a --pmc run of the read-request counters by size (TCC_EA0_RDREQ_32B_sum,
    _64B_sum, _128B_sum and TCC_EA0_RDREQ_sum) and one of the write-request
    counters (TCC_EA0_WRREQ_sum, TCC_EA0_WRREQ_64B_sum) -> HBM bytes per
    launch counted request by request (32, 64 or 128 bytes each), checked on
    the copy probe, whose bytes are known;
  * optionally a --pmc run of LDS counters (instructions, bank-conflict and
    active cycles).

The traffic quoted is the request-size count; FETCH_SIZE (which on gfx950
reads back about half of a copy's bytes) scaled by the copy probe is printed
beside it as a cross-check.

Writes a markdown summary and a JSON file with the per-launch traffic and the
hash of the kernel source it was measured on.

    python3 paper_2204_06666_amd/profile_summary.py --trace DIR --fetch DIR --write DIR \
        --rdreq DIR --wrreq DIR [--lds DIR] --fetch-log FILE \
        --out profiles/NAME.md --traffic profiles/NAME_traffic.json
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
    """Kernel statistics, and the mean duration of dispatches warmup ..
    warmup + steps - 1 of each summarised kernel ("|"-separated names), with
    the number of dispatches of the first."""
    stats = list(csv.DictReader(open(_one(os.path.join(trace_dir, "**", "*kernel_stats.csv")))))
    rows = list(csv.DictReader(open(_one(os.path.join(trace_dir, "**", "*kernel_trace.csv")))))
    means, count = {}, None
    for name in kernel.split("|"):
        ehyb = sorted((r for r in rows if name in r["Kernel_Name"]), key=lambda r: int(r["Start_Timestamp"]))
        dur = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) for r in ehyb]
        window = dur[warmup:warmup + steps]
        means[name] = statistics.mean(window) if window else None
        count = len(ehyb) if count is None else count
    return stats[:top], means, count


def pmc_values(pmc_dir, counter, kernel=KERNEL, scale=1024.0):
    """Mean per dispatch of `counter` for the EHYB kernel and for the copy
    probe (FETCH_SIZE / WRITE_SIZE are KiB: scale 1024; request counts: 1).
    `kernel` may name several kernels separated by "|" that each run once
    per product (the hub-row pre-pass and the product): "ehyb" is then the
    sum of their means, the count per product."""
    rows = list(csv.DictReader(open(_one(os.path.join(pmc_dir, "**", "*counter_collection.csv")))))
    names = kernel.split("|")
    per = {n: [] for n in names}
    copy = []
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        name = r["Kernel_Name"]
        v = float(r["Counter_Value"]) * scale
        if "probe_copy_kernel" in name:
            copy.append(v)
            continue
        for n in names:
            if n in name:
                per[n].append(v)
                break
    out = {}
    if all(per[n] for n in names):
        out["ehyb"] = sum(statistics.mean(per[n]) for n in names)
    if copy:
        out["copy"] = statistics.mean(copy)
    return out


def request_bytes(rd_dir, wr_dir, kernel):
    """Bytes read and written per dispatch, request by request."""
    n = {sz: pmc_values(rd_dir, f"TCC_EA0_RDREQ_{sz}B_sum", kernel, 1.0) for sz in (32, 64, 128)}
    tot = pmc_values(rd_dir, "TCC_EA0_RDREQ_sum", kernel, 1.0)
    wr = pmc_values(wr_dir, "TCC_EA0_WRREQ_sum", kernel, 1.0)
    wr64 = pmc_values(wr_dir, "TCC_EA0_WRREQ_64B_sum", kernel, 1.0)
    out = {}
    for key in ("ehyb", "copy"):
        reads = {sz: n[sz][key] for sz in n}
        out[key] = {"read_requests": {str(sz): round(v) for sz, v in reads.items()},
                    "read_requests_total": round(tot[key]),
                    "read_bytes": sum(sz * v for sz, v in reads.items()),
                    "write_requests": round(wr[key]), "write_requests_64B": round(wr64[key]),
                    "write_bytes": 64.0 * wr64[key] + 32.0 * (wr[key] - wr64[key])}
    return out


LDS_COUNTERS = ("SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE", "SQ_LDS_ADDR_CONFLICT", "SQ_WAVES",
                "SQ_BUSY_CYCLES", "SQ_WAVE_CYCLES", "SQ_WAIT_INST_LDS")


def lds_values(lds_dir, kernel):
    return {c: pmc_values(lds_dir, c, kernel, 1.0).get("ehyb") for c in LDS_COUNTERS}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--rdreq", required=True, help="--pmc run of the read-request counters by size")
    ap.add_argument("--wrreq", required=True, help="--pmc run of the write-request counters")
    ap.add_argument("--lds", default=None, help="--pmc run of the LDS counters")
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
    ap.add_argument("--log-tag", default="ehyb", help="product kind in the fetch log (ehyb, ehyb[f32], ...)")
    args = ap.parse_args()
    kernel = args.kernel

    stats, window_means, n_disp = trace_summary(args.trace, args.warmup, args.steps, kernel)
    window_ns = sum(window_means.values())
    log = open(args.fetch_log).read()
    m = re.search(re.escape(args.log_tag) + r" algorithmic_bytes=(\d+) copy_bytes_read=(\d+) copy_bytes_written=(\d+)",
                  log)
    algo, copy_r, copy_w = (int(g) for g in m.groups())
    fetch = pmc_values(args.fetch, "FETCH_SIZE", kernel)
    write = pmc_values(args.write, "WRITE_SIZE", kernel)
    f_scale = copy_r / fetch["copy"]
    w_scale = copy_w / write["copy"]
    fs_traffic = fetch["ehyb"] * f_scale + write["ehyb"] * w_scale
    req = request_bytes(args.rdreq, args.wrreq, kernel)
    e, c = req["ehyb"], req["copy"]
    traffic = e["read_bytes"] + e["write_bytes"]
    lds = lds_values(args.lds, kernel) if args.lds else None
    kh = kernel_source_hash()
    bench = None
    if args.bench_json:  # the JSON line bench.py prints (the last one in the file)
        bench = json.loads([ln for ln in open(args.bench_json) if ln.startswith("{")][-1])

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
    if len(window_means) == 1:
        lines += ["", f"Dispatches of `{kernel}` traced: {n_disp}. The benchmark's timed window is "
                      f"dispatches {args.warmup}..{args.warmup + args.steps - 1} (after {args.warmup} "
                      f"warm-up launches); their mean duration is **{window_ns / 1e3:.2f} us**."]
    else:
        each = ", ".join(f"`{k}` {v / 1e3:.2f} us" for k, v in window_means.items())
        lines += ["", f"One product is one dispatch of each of {len(window_means)} kernels ({n_disp} products "
                      f"traced). Over products {args.warmup}..{args.warmup + args.steps - 1} (after "
                      f"{args.warmup} warm-up products) their mean durations are {each}: "
                      f"**{window_ns / 1e3:.2f} us** of kernel time per product."]
    if bench:
        lines.append(f"bench.py measured {bench['roofline']['launch_us']} us per launch with HIP "
                     f"events in the same run ({bench['value']} GFLOP/s).")
        lines.append("The kernel's overall average above also includes every other launch of the same "
                     "kernel symbol in that run.")
    rq = e["read_requests"]
    lines += ["", "## HBM traffic per launch, request by request", "",
              "Read requests by size (TCC_EA0_RDREQ_32B/64B/128B_sum; their total TCC_EA0_RDREQ_sum) and "
              "write requests (TCC_EA0_WRREQ_sum, of which TCC_EA0_WRREQ_64B_sum are 64 bytes, the rest 32). "
              f"Check on the copy probe ({copy_r} bytes read, {copy_w} written): "
              f"{c['read_bytes']:.0f} bytes read ({c['read_bytes'] / copy_r:.4f}), "
              f"{c['write_bytes']:.0f} written ({c['write_bytes'] / copy_w:.4f}).", "",
              "| quantity | per launch |", "|---|---|",
              f"| read requests 32 / 64 / 128 B | {rq['32']} / {rq['64']} / {rq['128']} "
              f"(total {e['read_requests_total']}) |",
              f"| bytes read | {e['read_bytes']:.0f} |",
              f"| write requests (64 B of them) | {e['write_requests']} ({e['write_requests_64B']}) |",
              f"| bytes written | {e['write_bytes']:.0f} |",
              f"| **traffic per launch** | **{traffic:.0f}** |",
              f"| algorithmic bytes per launch | {algo} |",
              f"| traffic / algorithmic | {traffic / algo:.3f} |", "",
              "Cross-check (--pmc FETCH_SIZE, then --pmc WRITE_SIZE, each scaled by what it reads for the copy "
              f"probe: FETCH_SIZE x {f_scale:.4f}, WRITE_SIZE x {w_scale:.4f}): {fs_traffic:.0f} bytes per launch "
              f"({fs_traffic / algo:.3f} of the algorithmic bytes).", ""]
    if lds:
        bc, act = lds["SQ_LDS_BANK_CONFLICT"], lds["SQ_LDS_IDX_ACTIVE"]
        lines += ["## LDS counters per launch (--pmc " + " ".join(LDS_COUNTERS) + ")", "",
                  "| counter | value |", "|---|---|"]
        lines += [f"| {k} | {v:.0f} |" for k, v in lds.items() if v is not None]
        if bc is not None and act:
            lines += ["", f"Bank-conflict stall cycles per LDS-active cycle: {bc / act:.3f}."]
        lines.append("")
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    open(args.out, "w").write("\n".join(lines) + "\n")
    json.dump({"kernel": kernel, "workload": args.workload_name, "kernel_source_sha256_16": kh,
               "bytes_per_launch": round(traffic), "read_bytes": round(e["read_bytes"]),
               "write_bytes": round(e["write_bytes"]), "read_requests": rq,
               "read_requests_total": e["read_requests_total"], "write_requests": e["write_requests"],
               "write_requests_64B": e["write_requests_64B"],
               "copy_check": {"bytes_read": copy_r, "bytes_written": copy_w,
                              "read_bytes_counted": round(c["read_bytes"]),
                              "write_bytes_counted": round(c["write_bytes"])},
               "fetch_size_cross_check": {"bytes_per_launch": round(fs_traffic), "fetch_scale": f_scale,
                                          "write_scale": w_scale},
               "lds": lds, "algorithmic_bytes": algo,
               "timed_window_avg_us": round(window_ns / 1e3, 3)},
              open(args.traffic, "w"), indent=1)
    print(open(args.out).read())


if __name__ == "__main__":
    main()
