"""Turns rocprofv3 CSV output into the short text summaries kept with the
sources, and the per-launch HBM traffic table that bench.py reports.

    # kernel durations per dispatch (rocprofv3 --kernel-trace -f csv); for the
    # kernels matching --select, also the mean over dispatches skip..skip+take
    # of each (the timed steps of bench.py after its warmup)
    python -m paper_1502_05216_amd.profile_summary trace RUN_kernel_trace.csv \\
        --title "..." --command "..." --select "k_twofold<double" --skip 3 --take 20 \\
        --out profiles/NAME.md

    # HBM bytes from two counter runs of profile_run (FETCH_SIZE, WRITE_SIZE)
    python -m paper_1502_05216_amd.profile_summary traffic FETCH.csv WRITE.csv \\
        --n 67108864 --command-fetch "..." --command-write "..." \\
        --json profiles/traffic.json --out profiles/NAME.md

Both counters are reported in KiB per dispatch.  They are scaled by what the
same counter reads for a device-to-device copy of n binary64 values (n*8
bytes read and n*8 bytes written), run first in the same process.
"""
import argparse
import csv
import json
import os
import re
import sys
from collections import defaultdict

from ._build import source_hash

FN_NAMES = {0: "texp", 1: "texpm1", 2: "tlog", 3: "tlog1p"}
ARITH_NAMES = ["tadd", "tsub", "tmul", "tdiv", "tsqrt", "trenorm"]
IFACE_NAMES = ["pexp0", "texp0", "pexpm10", "texpm10", "plog0", "tlog0", "plog1p0", "tlog1p0",
               "pexp", "pexpm1", "tlogp", "plog", "tlog1pp", "plog1p"]


def short_name(kernel):
    """Readable name of a kernel from its demangled signature."""
    m = re.search(r"k_twofold<(double|float), (\d), (\d+), (\d+)(?:, (true|false))?>", kernel)
    if m:
        # "global tables": the instantiation that reads its tables in place
        return "k_twofold<%s,%s> ept%s pd%s%s" % (m.group(1), FN_NAMES[int(m.group(2))],
                                                  m.group(3), m.group(4),
                                                  " global tables" if m.group(5) == "true" else "")
    m = re.search(r"k_iface<(double|float), (\d+), (\d+)>", kernel)
    if m:
        return "k_iface<%s,%s> ept%s" % (m.group(1), IFACE_NAMES[int(m.group(2))], m.group(3))
    m = re.search(r"k_arith<(double|float), (\d), (\d+)>", kernel)
    if m:
        return "k_arith<%s,%s> ept%s" % (m.group(1), ARITH_NAMES[int(m.group(2))], m.group(3))
    m = re.search(r"k_backward<(double|float), (\d), (\d+)>", kernel)
    if m:
        return "k_backward<%s,%s> ept%s" % (m.group(1), FN_NAMES[int(m.group(2))], m.group(3))
    m = re.search(r"k_chain_bwd<(double|float), (\d+)>", kernel)
    if m:
        return "k_chain_bwd<%s> ept%s" % (m.group(1), m.group(2))
    m = re.search(r"(k_batch\w*)<?([\d, ]*)>?", kernel)
    if m:
        return m.group(1) + ("<%s>" % m.group(2) if m.group(2) else "")
    m = re.search(r"(k_onex)<(double|float), (\d)>", kernel)
    if m:
        return "k_onex<%s,%s>" % (m.group(2), m.group(3))
    return kernel.split("(")[0][:60]


def traffic_key(kernel):
    m = re.search(r"k_twofold<(double|float), (\d),", kernel)
    if m:
        return ("f64_" if m.group(1) == "double" else "f32_") + FN_NAMES[int(m.group(2))]
    m = re.search(r"k_iface<(double|float), (\d+),", kernel)
    if m:
        return ("f64_" if m.group(1) == "double" else "f32_") + IFACE_NAMES[int(m.group(2))]
    m = re.search(r"k_arith<(double|float), (\d),", kernel)
    if m:
        return ("f64_" if m.group(1) == "double" else "f32_") + ARITH_NAMES[int(m.group(2))]
    return None


def arrays_per_elem(name):
    """Arrays a kernel streams per element (inputs + outputs)."""
    if name in IFACE_NAMES[:8] or name in ("tsqrt", "trenorm"):
        return 3 if name in IFACE_NAMES[:8] else 4
    if name in ARITH_NAMES:
        return 6
    return 4


def stats(args):
    rows = list(csv.DictReader(open(args.csv)))
    lines = ["# %s" % args.title, "", "Command (from the repository root):", "",
             "    " + args.command.replace("\n", "\n    "), "",
             "Source hash of paper_1502_05216_amd/csrc: %s" % source_hash(), "",
             "| kernel | calls | average (us) | min (us) | max (us) | share |",
             "|---|---|---|---|---|---|"]
    for r in rows:
        name = r.get("Name") or r.get("KERNEL_NAME") or r.get("Kernel_Name")
        avg = float(r.get("AverageNs") or r.get("Average_ns") or 0) / 1e3
        mn = float(r.get("MinNs") or 0) / 1e3
        mx = float(r.get("MaxNs") or 0) / 1e3
        pct = float(r.get("Percentage") or 0)
        lines.append("| %s | %s | %.1f | %.1f | %.1f | %.1f%% |"
                     % (short_name(name), r.get("Calls"), avg, mn, mx, pct))
    if args.note:
        lines += ["", args.note]
    open(args.out, "w").write("\n".join(lines) + "\n")


def trace(args):
    groups = {}
    for r in csv.DictReader(open(args.csv)):
        key = (r["Kernel_Name"], int(r["Grid_Size_X"]), int(r["Workgroup_Size_X"]))
        g = groups.setdefault(key, {"d": [], "first": int(r["Dispatch_Id"]), "r": r})
        g["d"].append((int(r["Dispatch_Id"]),
                       (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3))
    lines = ["# %s" % args.title, "", "Command (from the repository root):", "",
             "    " + args.command.replace("\n", "\n    "), "",
             "Source hash of paper_1502_05216_amd/csrc: %s" % source_hash(), "",
             "Durations in microseconds, from the kernel trace (end - start of each dispatch).",
             "", "| kernel | grid x block | VGPR | LDS (B) | scratch (B) | dispatches | mean | "
             "median | min | max | mean of selected |", "|---|---|---|---|---|---|---|---|---|---|---|"]
    for (name, grid, block), g in sorted(groups.items(), key=lambda t: t[1]["first"]):
        d = [t for _, t in sorted(g["d"])]
        if len(d) < args.min_dispatches:
            continue
        if sum(d) / len(d) < args.min_mean and len(d) < args.keep_dispatches:
            continue
        ds = sorted(d)
        sel = ""
        if args.select and args.select in name:
            part = d[args.skip:args.skip + args.take]
            if part:
                sel = "%.1f (%d..%d)" % (sum(part) / len(part), args.skip + 1,
                                         args.skip + len(part))
        r = g["r"]
        lines.append("| %s | %d x %d | %s | %s | %s | %d | %.1f | %.1f | %.1f | %.1f | %s |"
                     % (short_name(name), grid // block, block, r["VGPR_Count"],
                        r["LDS_Block_Size"], r["Scratch_Size"], len(d), sum(d) / len(d),
                        ds[len(ds) // 2], ds[0], ds[-1], sel))
    if args.note:
        lines += ["", args.note]
    open(args.out, "w").write("\n".join(lines) + "\n")


def _per_kernel(path, counter):
    vals = defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            vals[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return vals


def traffic(args):
    fetch = _per_kernel(args.fetch_csv, "FETCH_SIZE")
    write = _per_kernel(args.write_csv, "WRITE_SIZE")
    copy_bytes = args.n * 8
    cf = [v for k, vs in fetch.items() if "copyBuffer" in k for v in vs]
    cw = [v for k, vs in write.items() if "copyBuffer" in k for v in vs]
    if not cf or not cw:
        sys.exit("no copy kernel in the counter runs")
    f_scale = copy_bytes / (cf[0] * 1024)
    w_scale = copy_bytes / (cw[0] * 1024)
    h = source_hash()
    out = {"src_hash": h, "n": args.n, "copy_bytes": copy_bytes,
           "copy_fetch_kib": cf[0], "copy_write_kib": cw[0],
           "fetch_scale": f_scale, "write_scale": w_scale, "kernels": {}}
    lines = ["# HBM traffic per launch of the streaming kernels, 2^26 elements (MI355X)", "",
             "Counter runs (from the repository root; one counter per run):", "",
             "    " + args.command_fetch, "    " + args.command_write, "",
             "Source hash of paper_1502_05216_amd/csrc: %s" % h, "",
             "Scale: a device-to-device copy of %d bytes reads FETCH_SIZE %.0f KiB and "
             "WRITE_SIZE %.0f KiB, so FETCH_SIZE is multiplied by %.3f and WRITE_SIZE by %.3f."
             % (copy_bytes, cf[0], cw[0], f_scale, w_scale), "",
             "| kernel | dispatches | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | scaled bytes | "
             "algorithmic bytes | ratio |", "|---|---|---|---|---|---|---|"]
    for k in sorted(fetch):
        key = traffic_key(k)
        if key is None or k not in write:
            continue
        fk = sum(fetch[k]) / len(fetch[k])
        wk = sum(write[k]) / len(write[k])
        b = fk * 1024 * f_scale + wk * 1024 * w_scale
        alg = args.n * arrays_per_elem(key.split("_", 1)[1]) * (8 if key.startswith("f64") else 4)
        out["kernels"][key] = {"src_hash": h, "n": args.n, "bytes_per_launch": b,
                               "algorithmic_bytes": alg, "fetch_kib": fk, "write_kib": wk,
                               "dispatches": len(fetch[k])}
        lines.append("| %s | %d | %.0f | %.0f | %.4g | %.4g | %.3f |"
                     % (short_name(k), len(fetch[k]), fk, wk, b, alg, b / alg))
    json.dump(out, open(args.json, "w"), indent=1)
    open(args.out, "w").write("\n".join(lines) + "\n")


def _counters(path):
    """{kernel: {counter: [values]}} and {kernel: [durations in s]} of a
    rocprofv3 counter-collection CSV (one row per dispatch and counter)."""
    vals = defaultdict(lambda: defaultdict(list))
    dur = defaultdict(dict)
    for r in csv.DictReader(open(path)):
        k = r["Kernel_Name"]
        vals[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
        dur[k][r["Dispatch_Id"]] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    return vals, {k: list(v.values()) for k, v in dur.items()}


def valu(args):
    """VALU instruction counts of the twofold-function kernels: instructions
    per element, the clock (GRBM_GUI_ACTIVE counts busy cycles of each XCD),
    the fraction of VALU issue slots used (a wave64 VALU instruction occupies a
    SIMD16 for 4 cycles: at most one per CU per cycle), and from the second run
    the executed FP64 instruction mix against the oracle's algorithmic count."""
    a, da = _counters(args.csv_a)
    b, _ = _counters(args.csv_b) if args.csv_b else ({}, {})
    opc = json.load(open(args.opcounts))
    mean = lambda v: sum(v) / len(v)
    lines = ["# VALU instruction counters of the twofold-function kernels, 2^26 elements (MI355X)",
             "", "Counter runs (from the repository root):", "", "    " + args.command_a]
    if args.csv_b:
        lines.append("    " + args.command_b)
    lines += ["", "Source hash of paper_1502_05216_amd/csrc: %s" % source_hash(), "",
              "VALU/elem = SQ_INSTS_VALU x 64 / n (wave instructions to lane instructions). "
              "Clock = GRBM_GUI_ACTIVE / (%d XCDs x dispatch duration). Issue slots used = "
              "SQ_INSTS_VALU / (%d CUs x cycles): a wave64 instruction takes a SIMD16 four "
              "cycles at the FP64 rate, so a CU issues at most one per cycle; 32-bit "
              "instructions can issue faster, so the column is an upper bound for the binary64 "
              "kernels and is left out for binary32. FP64 columns: "
              "SQ_INSTS_VALU_{ADD,MUL,FMA}_F64 x 64 / n; executed flops count FMA as 2; the "
              "algorithmic counts are the oracle's (tests/golden/opcounts.json)."
              % (args.xcds, args.cus), "",
              "| kernel | dispatches | us | clock (GHz) | VALU/elem | FP64-rate slots used | "
              "alg. ops/elem | F64 add | F64 mul | F64 fma | executed flops/elem | "
              "alg. flops/elem |", "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for k in sorted(a):
        m = re.search(r"k_twofold<(double|float), (\d),", k)
        if not m or "SQ_INSTS_VALU" not in a[k]:
            continue
        dts = "f64" if m.group(1) == "double" else "f32"
        fn = FN_NAMES[int(m.group(2))]
        ins = mean(a[k]["SQ_INSTS_VALU"])
        d = mean(da[k])
        cyc = mean(a[k]["GRBM_GUI_ACTIVE"]) / args.xcds
        row = [short_name(k), str(len(da[k])), "%.1f" % (d * 1e6), "%.2f" % (cyc / d / 1e9),
               "%.1f" % (ins * 64 / args.n),
               "%.2f" % (ins / (args.cus * cyc)) if dts == "f64" else "",
               "%.1f" % opc[dts][fn]["ops"]]
        if k in b and "SQ_INSTS_VALU_FMA_F64" in b[k]:
            ad, mu, fm = (mean(b[k]["SQ_INSTS_VALU_%s_F64" % t]) * 64 / args.n
                          for t in ("ADD", "MUL", "FMA"))
            row += ["%.1f" % ad, "%.1f" % mu, "%.1f" % fm, "%.1f" % (ad + mu + 2 * fm)]
        else:
            row += ["", "", "", ""]
        row.append("%.1f" % opc[dts][fn]["flops"])
        lines.append("| " + " | ".join(row) + " |")
    if args.note:
        lines += ["", args.note]
    open(args.out, "w").write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--title", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--note", default="")
    s.add_argument("--out", required=True)
    s = sub.add_parser("trace")
    s.add_argument("csv")
    s.add_argument("--title", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--select", default="")
    s.add_argument("--skip", type=int, default=0)
    s.add_argument("--take", type=int, default=1 << 30)
    s.add_argument("--min-dispatches", type=int, default=2)
    s.add_argument("--min-mean", type=float, default=0.0, help="drop groups with a smaller "
                   "mean duration (us), e.g. the small per-array launches")
    s.add_argument("--keep-dispatches", type=int, default=1 << 30,
                   help="keep groups with at least this many dispatches whatever their mean")
    s.add_argument("--note", default="")
    s.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("--n", type=int, default=1 << 26)
    t.add_argument("--command-fetch", required=True)
    t.add_argument("--command-write", required=True)
    t.add_argument("--json", required=True)
    t.add_argument("--out", required=True)
    v = sub.add_parser("valu")
    v.add_argument("csv_a", help="counter CSV with SQ_INSTS_VALU and GRBM_GUI_ACTIVE")
    v.add_argument("--csv-b", default="", help="counter CSV with SQ_INSTS_VALU_*_F64")
    v.add_argument("--n", type=int, default=1 << 26)
    v.add_argument("--xcds", type=int, default=8)
    v.add_argument("--cus", type=int, default=256)
    v.add_argument("--opcounts", default=os.path.join(os.path.dirname(os.path.dirname(
        os.path.abspath(__file__))), "tests", "golden", "opcounts.json"))
    v.add_argument("--command-a", required=True)
    v.add_argument("--command-b", default="")
    v.add_argument("--note", default="")
    v.add_argument("--out", required=True)
    args = ap.parse_args()
    {"stats": stats, "trace": trace, "traffic": traffic, "valu": valu}[args.cmd](args)


if __name__ == "__main__":
    main()
