"""Condense rocprofv3 CSV output into the short text / JSON summaries kept
with the measurements.

    python -m paper_2208_08038_amd.profile_summary stats KERNEL_STATS_CSV \
        --command "rocprofv3 ... -- python3 bench.py ..." --out FILE [--top 12]

writes the per-kernel call count and average / total duration table of a
`rocprofv3 --kernel-trace --stats --output-format csv` run.

    python -m paper_2208_08038_amd.profile_summary traffic \
        --fetch CSV --write CSV --copy-fetch CSV --copy-write CSV \
        --copy-bytes N --kernel NAME --workload KEY --out FILE.json

turns two `--pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs of the bench
(counter values in KiB per dispatch) into HBM bytes per dispatch of one
kernel, each scaled by what the same counter reads for a plain device copy
of N bytes (which must fetch N and write N bytes); with --req-read /
--req-write (and the copy's), also the bytes counted by TCC request size.

    python -m paper_2208_08038_amd.profile_summary counters CSV... \
        --kernel NAME --pairs N --command "..." --out FILE

writes the per-dispatch means of the SQ counters of `--pmc` runs, with the
VALU issue rate and instructions per ion + electron pair.
"""
import argparse
import csv
import hashlib
import json
import os
import re
import statistics

PKG = os.path.dirname(os.path.abspath(__file__))

# sources whose change invalidates a stored traffic measurement of the
# particle kernel
KERNEL_SOURCES = ["cycle.h", "tiled.hip", "tiled.h", "pic_internal.h"]


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(PKG, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short_name(name):
    """Kernel name without namespaces and argument list."""
    n = name.strip().strip('"').replace("(anonymous namespace)::", "")
    depth, cut = 0, len(n)
    for i, ch in enumerate(n):  # cut at the argument list's '(' (outside <>)
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0 and i > 0:
            cut = i
            break
    n = n[:cut]
    n = re.sub(r"^void ", "", n).replace("pic::", "")
    return n if len(n) <= 96 else n[:93] + "..."


def read_rows(path):
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def stats(args):
    rows = read_rows(args.csv)
    out = []
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out.append(f"# rocprofv3 kernel statistics: {args.title}")
    out.append(f"# command: {args.command}")
    out.append(f"# GPU kernel time in the profile: {total / 1e6:.3f} ms")
    out.append(f"{'calls':>6} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'total_ms':>10} {'pct':>6}  kernel")
    for r in rows[: args.top]:
        out.append(f"{int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.2f} "
                   f"{float(r['MinNs']) / 1e3:10.2f} {float(r['MaxNs']) / 1e3:10.2f} "
                   f"{float(r['TotalDurationNs']) / 1e6:10.3f} {float(r['Percentage']):6.2f}  "
                   f"{short_name(r['Name'])}")
    if args.note:
        out.append("")
        out.extend(f"# {line}" for line in args.note)
    text = "\n".join(out) + "\n"
    with open(args.out, "w") as fh:
        fh.write(text)
    print(text, end="")


def counter_per_dispatch(path, counter, match, largest_grid=False):
    """Mean over the dispatches of kernels whose name contains `match` of
    the named counter (summed over the agent's instances); with
    `largest_grid` only the dispatches of the largest grid count (a copy
    kernel also serves small copies)."""
    per, grid = {}, {}
    for r in read_rows(path):
        if r["Counter_Name"] != counter or match not in r["Kernel_Name"]:
            continue
        d = r["Dispatch_Id"]
        per[d] = per.get(d, 0.0) + float(r["Counter_Value"])
        grid[d] = int(r["Grid_Size"])
    if largest_grid and grid:
        gmax = max(grid.values())
        per = {d: v for d, v in per.items() if grid[d] == gmax}
    if not per:
        raise SystemExit(f"{path}: no {counter} rows for kernels matching {match!r}")
    vals = list(per.values())
    return statistics.mean(vals), len(vals), (statistics.pstdev(vals) if len(vals) > 1 else 0.0)


def traffic(args):
    kib = 1024.0
    copy_kernel = args.copy_kernel
    cf, ncf, _ = counter_per_dispatch(args.copy_fetch, "FETCH_SIZE", copy_kernel, True)
    cw, ncw, _ = counter_per_dispatch(args.copy_write, "WRITE_SIZE", copy_kernel, True)
    f_fetch = args.copy_bytes / (cf * kib)
    f_write = args.copy_bytes / (cw * kib)
    kf, nkf, sf = counter_per_dispatch(args.fetch, "FETCH_SIZE", args.kernel)
    kw, nkw, sw = counter_per_dispatch(args.write, "WRITE_SIZE", args.kernel)
    res = {
        "kernel": args.kernel,
        "workload": args.workload,
        "kernel_source_hash": kernel_source_hash(),
        "fetch_kib_per_dispatch": kf, "write_kib_per_dispatch": kw,
        "dispatches": [nkf, nkw], "fetch_kib_stdev": sf, "write_kib_stdev": sw,
        "copy_kernel": short_name(copy_kernel), "copy_bytes": args.copy_bytes,
        "copy_dispatches": [ncf, ncw],
        "copy_fetch_kib": cf, "copy_write_kib": cw,
        "scale_fetch": f_fetch, "scale_write": f_write,
        "fetch_bytes_per_launch": kf * kib * f_fetch,
        "write_bytes_per_launch": kw * kib * f_write,
        "bytes_per_launch": kf * kib * f_fetch + kw * kib * f_write,
        "commands": args.command or [],
    }
    if args.req_read and args.req_write:
        res["by_request_size"] = request_bytes(args.req_read, args.req_write, args.kernel)
        res["by_request_size_copy"] = request_bytes(args.req_copy_read, args.req_copy_write,
                                                    copy_kernel, True)
    with open(args.out, "w") as fh:
        json.dump(res, fh, indent=1)
        fh.write("\n")
    print(json.dumps(res, indent=1))


def request_bytes(t1, t2, kernel, largest_grid=False):
    """HBM-side bytes per dispatch from the TCC request counters: reads
    32 / 64 / 128 B by request size (TCC_EA0_RDREQ_{32B,64B,128B}_sum),
    writes 64 B (TCC_EA0_WRREQ_64B_sum) or 32 B (the rest of
    TCC_EA0_WRREQ_sum)."""
    r32, n, _ = counter_per_dispatch(t1, "TCC_EA0_RDREQ_32B_sum", kernel, largest_grid)
    r64, _, _ = counter_per_dispatch(t1, "TCC_EA0_RDREQ_64B_sum", kernel, largest_grid)
    r128, _, _ = counter_per_dispatch(t1, "TCC_EA0_RDREQ_128B_sum", kernel, largest_grid)
    w, _, _ = counter_per_dispatch(t2, "TCC_EA0_WRREQ_sum", kernel, largest_grid)
    w64, _, _ = counter_per_dispatch(t2, "TCC_EA0_WRREQ_64B_sum", kernel, largest_grid)
    return {"read_requests_32_64_128": [r32, r64, r128], "write_requests_all_64": [w, w64],
            "read_bytes": 32 * r32 + 64 * r64 + 128 * r128,
            "write_bytes": 64 * w64 + 32 * (w - w64), "dispatches": n}


def counters(args):
    """Mean per dispatch of every counter in the CSVs for kernels matching
    --kernel, with the derived issue rates."""
    sums, durs = {}, {}
    for path in args.csv:
        per, dur = {}, {}
        for r in read_rows(path):
            if args.kernel not in r["Kernel_Name"]:
                continue
            d = r["Dispatch_Id"]
            per.setdefault(d, {})
            per[d][r["Counter_Name"]] = per[d].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
            dur[d] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
        for d, cs in per.items():
            for k, v in cs.items():
                sums.setdefault(k, []).append(v)
        durs.update({(path, d): t for d, t in dur.items()})
    if not sums:
        raise SystemExit(f"no counter rows for kernels matching {args.kernel!r}")
    m = {k: statistics.mean(v) for k, v in sums.items()}
    t = statistics.mean(durs.values())
    out = [f"# rocprofv3 counters: {args.title}",
           f"# kernel source hash: {kernel_source_hash()}",
           "# commands (each pass its own run):"]
    out += [f"#   {c}" for c in args.command or []]
    out.append(f"# values: mean per dispatch of {short_name(args.kernel)}, summed over the "
               f"agent's counter instances; {len(durs)} dispatches, mean duration under "
               f"counters {t * 1e6:.1f} us")
    out.append(f"# per pair: wave instructions x 64 / {args.pairs:.0f} (ions of one dispatch, "
               "each with one electron)")
    out.append("")
    for k in sorted(m):
        out.append(f"    {k:28s} {m[k]:.4e}")
    per_pair = lambda k: m.get(k, 0.0) * 64.0 / args.pairs
    out.append("")
    if "SQ_INSTS_VALU" in m:
        busy = m["SQ_INSTS_VALU"] / (t * args.clock * args.cus)
        out.append(f"    VALU issue (one wave instruction per CU per clock) {busy:.2f}")
        out.append(f"    VALU instructions per pair        {per_pair('SQ_INSTS_VALU'):8.0f}")
    groups = [("FP32 FMA+MUL+ADD", ["SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_MUL_F32",
                                     "SQ_INSTS_VALU_ADD_F32"]),
              ("FP64 FMA+MUL+ADD", ["SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_MUL_F64",
                                     "SQ_INSTS_VALU_ADD_F64"]),
              ("transcendental", ["SQ_INSTS_VALU_TRANS_F32", "SQ_INSTS_VALU_TRANS_F64"]),
              ("INT32", ["SQ_INSTS_VALU_INT32"]), ("INT64", ["SQ_INSTS_VALU_INT64"]),
              ("CVT", ["SQ_INSTS_VALU_CVT"]), ("LDS", ["SQ_INSTS_LDS"]),
              ("SALU", ["SQ_INSTS_SALU"]), ("VMEM", ["SQ_INSTS_VMEM"])]
    for name, ks in groups:
        if any(k in m for k in ks):
            out.append(f"    {name + ' per pair':34s} {sum(per_pair(k) for k in ks):8.0f}")
    if "SQ_LDS_BANK_CONFLICT" in m and m.get("SQ_ACTIVE_INST_LDS"):
        out.append(f"    LDS bank-conflict / LDS-active cycles  "
                   f"{m['SQ_LDS_BANK_CONFLICT'] / m['SQ_ACTIVE_INST_LDS']:.2f}")
    if args.note:
        out.append("")
        out.extend(f"# {line}" for line in args.note)
    text = "\n".join(out) + "\n"
    with open(args.out, "w") as fh:
        fh.write(text)
    print(text, end="")


def main():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="mode", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--command", required=True)
    s.add_argument("--title", default="")
    s.add_argument("--out", required=True)
    s.add_argument("--top", type=int, default=12)
    s.add_argument("--note", action="append")
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        t.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--copy-kernel", default="__amd_rocclr_copyBuffer",
                   help="name (substring) of the copy kernel in the calibration runs")
    t.add_argument("--kernel", required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--command", action="append")
    t.add_argument("--out", required=True)
    for k in ("req_read", "req_write", "req_copy_read", "req_copy_write"):
        t.add_argument("--" + k.replace("_", "-"), dest=k, default=None,
                       help="TCC request-count runs (reads: TCC_EA0_RDREQ_{32B,64B,128B}_sum; "
                            "writes: TCC_EA0_WRREQ_sum, TCC_EA0_WRREQ_64B_sum)")
    c = sub.add_parser("counters")
    c.add_argument("csv", nargs="+")
    c.add_argument("--kernel", required=True)
    c.add_argument("--pairs", type=float, required=True)
    c.add_argument("--clock", type=float, default=2.4e9)
    c.add_argument("--cus", type=int, default=256)
    c.add_argument("--title", default="")
    c.add_argument("--command", action="append")
    c.add_argument("--note", action="append")
    c.add_argument("--out", required=True)
    a = ap.parse_args()
    {"stats": stats, "traffic": traffic, "counters": counters}[a.mode](a)


if __name__ == "__main__":
    main()
