"""Summaries of rocprofv3 CSV output for the kernels of libeslb.

    python -m paper_2403_13406_amd.profiling stats <kernel_stats.csv>
    python -m paper_2403_13406_amd.profiling traffic --fetch <fetch counter_collection.csv>
        --write <write counter_collection.csv> --kernel k_stage --copy-bytes N --workload TAG --out FILE.json
    python -m paper_2403_13406_amd.profiling valu --csv <counter_collection.csv> --kernel k_stage
        --nodes N --workload TAG --out FILE.json [--kernel-us T]

HBM traffic of a kernel: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) averaged over
the kernel's dispatches, each scaled by known-bytes / counter-reading of a plain
device-to-device copy of N bytes profiled in the same run (the copy's own
FETCH_SIZE and WRITE_SIZE should read N bytes each).
"""
import argparse
import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_KERNEL_HINTS = ("copyBuffer", "copy_kernel", "elementwise_kernel")


def source_hash():
    """Hash of the HIP sources: a counter record is valid only for the kernels it measured."""
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_stats(path):
    rows = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            rows.append((r["Name"], int(r["Calls"]), float(r["AverageNs"]), float(r["Percentage"])))
    return rows


def counters(path):
    """{kernel name: {counter: [values per dispatch]}} from a counter_collection.csv."""
    out = defaultdict(lambda: defaultdict(list))
    with open(path) as fh:
        for r in csv.DictReader(fh):
            out[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return out


def _pick(table, needle):
    names = [n for n in table if needle in n]
    if not names:
        raise SystemExit("no kernel matching %r in %s" % (needle, sorted(table)))
    return names[0]


def _copy(table):
    for hint in COPY_KERNEL_HINTS:
        names = [n for n in table if hint in n]
        if names:
            return names[0]
    raise SystemExit("no copy kernel found for the calibration")


def traffic(fetch_csv, write_csv, kernel, copy_bytes):
    f = counters(fetch_csv)
    w = counters(write_csv)
    kf, kw = _pick(f, kernel), _pick(w, kernel)
    cf, cw = _copy(f), _copy(w)
    mean = lambda v: sum(v) / len(v)
    fetch_kib = mean(f[kf]["FETCH_SIZE"])
    write_kib = mean(w[kw]["WRITE_SIZE"])
    # the copy is the largest dispatch of its kernel (the calibration copy)
    copy_fetch_kib = max(f[cf]["FETCH_SIZE"])
    copy_write_kib = max(w[cw]["WRITE_SIZE"])
    sf = copy_bytes / (copy_fetch_kib * 1024.0)
    sw = copy_bytes / (copy_write_kib * 1024.0)
    return {
        "kernel": kf,
        "dispatches": len(f[kf]["FETCH_SIZE"]),
        "fetch_kib_per_launch": fetch_kib,
        "write_kib_per_launch": write_kib,
        "copy_kernel": cf,
        "copy_bytes": copy_bytes,
        "copy_fetch_kib": copy_fetch_kib,
        "copy_write_kib": copy_write_kib,
        "scale_fetch": sf,
        "scale_write": sw,
        "bytes_per_launch": fetch_kib * 1024.0 * sf + write_kib * 1024.0 * sw,
    }


XCDS = 8  # GRBM_GUI_ACTIVE is summed over the eight accelerator complex dies of an MI355X


def valu(valu_csv, kernel, nodes, kernel_us=None):
    """FP64 VALU instructions per node of a kernel (SQ_INSTS_VALU_*_F64 count wave instructions).

    With GRBM_GUI_ACTIVE in the same pass and the kernel's average duration (from a
    kernel trace), the clock the chip held: busy cycles per die / duration."""
    c = counters(valu_csv)
    k = _pick(c, kernel)
    mean = lambda v: sum(v) / len(v)
    per = {name: mean(vals) * 64.0 / nodes for name, vals in c[k].items() if name.startswith("SQ_INSTS")}
    flop = (per.get("SQ_INSTS_VALU_ADD_F64", 0.0) + per.get("SQ_INSTS_VALU_MUL_F64", 0.0)
            + 2.0 * per.get("SQ_INSTS_VALU_FMA_F64", 0.0) + per.get("SQ_INSTS_VALU_TRANS_F64", 0.0))
    rec = {"kernel": k, "dispatches": len(next(iter(c[k].values()))), "nodes": nodes,
           "lane_instructions_per_node": per, "fp64_flop_per_node": flop}
    if "GRBM_GUI_ACTIVE" in c[k]:
        cyc = mean(c[k]["GRBM_GUI_ACTIVE"]) / XCDS
        rec["gui_active_cycles_per_die"] = cyc
        if kernel_us:
            rec["kernel_us"] = kernel_us
            rec["clock_ghz"] = round(cyc / (kernel_us * 1e3), 3)
    return rec


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", default="k_stage")
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--out", required=True)
    v = sub.add_parser("valu")
    v.add_argument("--csv", required=True)
    v.add_argument("--kernel", default="k_stage")
    v.add_argument("--nodes", type=int, required=True)
    v.add_argument("--workload", required=True)
    v.add_argument("--out", required=True)
    v.add_argument("--kernel-us", type=float, default=None,
                   help="average duration of the kernel (trace of the same command), for the clock")
    a = ap.parse_args(argv)
    if a.cmd == "valu":
        rec = valu(a.csv, a.kernel, a.nodes, a.kernel_us)
        rec["workload"] = a.workload
        rec["source_hash"] = source_hash()
        with open(a.out, "w") as fh:
            json.dump(rec, fh, indent=1)
        print(json.dumps(rec, indent=1))
        return 0
    if a.cmd == "stats":
        print("%-100s %7s %14s %8s" % ("kernel", "calls", "avg_us", "pct"))
        for name, calls, avg, pct in kernel_stats(a.csv):
            print("%-100s %7d %14.2f %8.3f" % (name[:100], calls, avg / 1e3, pct))
        return 0
    rec = traffic(a.fetch, a.write, a.kernel, a.copy_bytes)
    rec["workload"] = a.workload
    rec["source_hash"] = source_hash()
    with open(a.out, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec, indent=1))
    return 0


if __name__ == "__main__":
    sys.exit(main())
