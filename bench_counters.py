"""Turn rocprofv3 output of `bench.py` runs on one workload into the counter
summary `profiles/<workload>_counters.txt` that bench.py reads back, or, with
--kernel-stats, one `--kernel-trace --stats` run into the kernel time summary
`profiles/<workload>_kernel_stats.txt`.

Inputs: the CSV directories of one `--kernel-trace --stats` run and of four
`--pmc` runs (FETCH_SIZE; WRITE_SIZE; TCC_HIT_sum TCC_MISS_sum; SQ_INSTS_VALU
SQ_WAVES), each of the same bench.py command with `--copy-probe-mib 256`.
Per kernel: mean counter value per dispatch, and its mean duration from the
trace.  HBM bytes per dispatch = FETCH_SIZE x f + WRITE_SIZE x w (KiB x 1024),
with f and w the factors that make the 256 MiB copy read and write 256 MiB;
L2 hit rate = hits / (hits + misses); VALU issue fraction = VALU wave
instructions / duration / the issue peak (256 CUs x 4 SIMDs x 2.4 GHz / 4
cycles per wave64 instruction).  The Infinity Cache (MALL) has no counter in
rocprofv3 on gfx950, so its hit rate is '-'.

    python bench_counters.py --workload W --trace D0 --fetch D1 --write D2 --tcc D3 --sq D4 \\
        --command "..." > profiles/W_counters.txt
    python bench_counters.py --kernel-stats --workload W --trace D0 --command "..." \\
        [--note "..."]... > profiles/W_kernel_stats.txt
"""
import argparse
import collections
import csv
import glob
import hashlib
import os

ROOT = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(ROOT, "paper_2004_08475_amd", "csrc", "amriso.hip")
VALU_PEAK = 256 * 4 * 2.4e9 / 4  # wave64 instructions per second
COPY_KIB = 256 * 1024


def short_name(k):
    k = k.replace("(anonymous namespace)::", "")
    if k.startswith("void "):
        k = k[len("void "):]
    depth, out = 0, []
    for ch in k:  # the name up to its argument list (template arguments kept)
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            break
        out.append(ch)
    return "".join(out).strip()


def one_csv(d, suffix):
    paths = glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)
    if len(paths) != 1:
        raise SystemExit("expected one *%s under %s, found %d" % (suffix, d, len(paths)))
    return paths[0]


def counters(d):
    acc = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(set)
    with open(one_csv(d, "counter_collection.csv")) as fh:
        for row in csv.DictReader(fh):
            k = short_name(row["Kernel_Name"])
            disp[k].add(row["Dispatch_Id"])
            acc[k][row["Counter_Name"]] += float(row["Counter_Value"])
    return {k: {c: v / len(disp[k]) for c, v in cs.items()} for k, cs in acc.items()}


def durations(d):
    out = {}
    with open(one_csv(d, "kernel_stats.csv")) as fh:
        for row in csv.DictReader(fh):
            out[short_name(row["Name"])] = (int(row["Calls"]), float(row["AverageNs"]) / 1e3)
    return out


def stats_rows(d):
    """The library's kernels (names starting k_) of one trace's stats CSV:
    (name, calls, total, average, min, max), durations in us, longest total
    first."""
    rows = []
    with open(one_csv(d, "kernel_stats.csv")) as fh:
        for row in csv.DictReader(fh):
            k = short_name(row["Name"])
            if k.startswith("k_"):
                rows.append((k, int(row["Calls"]), float(row["TotalDurationNs"]) / 1e3,
                             float(row["AverageNs"]) / 1e3, float(row["MinNs"]) / 1e3, float(row["MaxNs"]) / 1e3))
    return sorted(rows, key=lambda r: -r[2])


def kernel_stats(args):
    print("# rocprofv3 kernel trace summary, one MI355X (ROCm 7.2): %s" % args.workload)
    print("# Command (repo root $R; run from /tmp with TMPDIR=/tmp):")
    for ln in args.command.splitlines():
        print("#   " + ln)
    print("#   then: python $R/bench_counters.py --kernel-stats --workload %s --trace <out> --command ... --note ..."
          % args.workload)
    for ln in args.note:
        print("# " + ln)
    print("# From run_kernel_stats.csv: the library's kernels (name without arguments), calls, durations in us.")
    print("%-30s %5s %12s %12s %12s %12s" % ("kernel", "calls", "total_us", "avg_us", "min_us", "max_us"))
    for k, calls, tot, avg, lo, hi in stats_rows(args.trace):
        print("%-30s %5d %12.1f %12.2f %12.2f %12.2f" % (k, calls, tot, avg, lo, hi))


def copy_kernel(c):
    """The probe of `bench.py --copy-probe-mib 256` (torch.mul by 1 into a
    second tensor), the run's only float multiply kernel."""
    ks = [k for k in c if "MulFunctor<float>" in k]
    if len(ks) != 1:
        raise SystemExit("no unique copy-probe kernel among %s" % sorted(c))
    return ks[0]


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--kernel-stats", action="store_true", help="summarise the --trace run's kernel times only")
    for a in ("workload", "trace", "command"):
        ap.add_argument("--" + a, required=True)
    for a in ("fetch", "write", "tcc", "sq"):
        ap.add_argument("--" + a)
    ap.add_argument("--note", action="append", default=[], help="a line describing the run (kernel stats)")
    args = ap.parse_args()
    if args.kernel_stats:
        kernel_stats(args)
        return
    missing = [a for a in ("fetch", "write", "tcc", "sq") if getattr(args, a) is None]
    if missing:
        ap.error("counter summaries need --" + ", --".join(missing))
    dur = durations(args.trace)
    fetch, write, tcc, sq = (counters(getattr(args, a)) for a in ("fetch", "write", "tcc", "sq"))
    ck = copy_kernel(fetch)
    f_scale = COPY_KIB / fetch[ck]["FETCH_SIZE"]
    w_scale = COPY_KIB / write[copy_kernel(write)]["WRITE_SIZE"]
    src = hashlib.sha256(open(SOURCE, "rb").read()).hexdigest()
    print("# rocprofv3 counters of the library's kernels on workload %s, one MI355X (ROCm 7.2)." % args.workload)
    print("# Commands (repo root $R; run from /tmp with TMPDIR=/tmp), one rocprofv3 run each:")
    for ln in args.command.splitlines():
        print("#   " + ln)
    print("# Per dispatch, averaged over each kernel's dispatches.  Scale from the 256 MiB copy probe "
          "(%s): bytes = FETCH_SIZE x %.3f + WRITE_SIZE x %.3f (KiB x 1024)." % (ck[:60], f_scale, w_scale))
    print("# l2_hit = TCC_HIT / (TCC_HIT + TCC_MISS); valu_issue = SQ_INSTS_VALU / avg duration / %.4g; "
          "mall_hit '-': no Infinity Cache counter on gfx950." % VALU_PEAK)
    print("# The line 'source_sha256' is the hash of paper_2004_08475_amd/csrc/amriso.hip these were taken with;")
    print("# bench.py uses the figures only while the source still has that hash.")
    print("source_sha256 %s" % src)
    for k in sorted(dur, key=lambda k: -dur[k][0] * dur[k][1]):
        if not k.startswith("k_") or k not in fetch or k not in write:
            continue
        calls, us = dur[k]
        fb = fetch[k]["FETCH_SIZE"] * f_scale * 1024
        wb = write[k]["WRITE_SIZE"] * w_scale * 1024
        t = tcc.get(k, {})
        h, m = t.get("TCC_HIT_sum"), t.get("TCC_MISS_sum")
        l2 = "%.4f" % (h / (h + m)) if h is not None and m is not None and h + m > 0 else "-"
        v = sq.get(k, {}).get("SQ_INSTS_VALU")
        valu = "%.4f" % (v / (us * 1e-6) / VALU_PEAK) if v is not None and us > 0 else "-"
        waves = sq.get(k, {}).get("SQ_WAVES")
        print("kernel %s | traffic_bytes %.6g fetch_bytes %.6g write_bytes %.6g l2_hit %s mall_hit - "
              "valu_issue %s avg_us %.2f calls %d waves %s" % (k, fb + wb, fb, wb, l2, valu, us, calls,
                                                                 "%.0f" % waves if waves is not None else "-"))


if __name__ == "__main__":
    main()
