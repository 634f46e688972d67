"""Summaries of rocprofv3 output behind the benchmark's roofline figures.

    python -m paper_2109_00214_amd.profiling stats DIR CMD...
        kernel-trace stats (rocprofv3 --kernel-trace --stats) -> text table
    python -m paper_2109_00214_amd.profiling copy BYTES
        a plain device copy of BYTES bytes, three times (the counter calibration run)
    python -m paper_2109_00214_amd.profiling traffic FETCH_DIR WRITE_DIR CAL_FETCH_DIR
                                               CAL_WRITE_DIR CAL_BYTES BENCH_LOG SKIP CMD...
        two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) of
        CMD, each scaled by what the same counter reads for the copy run -> text table
        ending in one "stage" line per roofline stage, which bench.py reads.  BENCH_LOG
        is CMD's output (a bench.py run): its mean particles per timed step turn bytes
        per dispatch into bytes per particle; the first SKIP dispatches of every kernel
        (the warm-up steps, once per step for the stage kernels) are left out.

A "stage" line records the source files of its kernel by SHA-256, so a kernel
changed after its counters were taken reports no traffic.
"""
import csv
import glob
import hashlib
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
# stage -> (kernel name, sources that define it)
STAGE_KERNELS = {
    "push": ("pd::k_push<double>", ("csrc/k_pic.hip", "csrc/pd_internal.h")),
}


def source_digest(files):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(HERE, f), "rb").read())
    return h.hexdigest()[:16]


def stage_line(stage, fetch_b, write_b, particles):
    """The summary line of one roofline stage (read back by read_traffic)."""
    k, files = STAGE_KERNELS[stage]
    return "stage %s %s %.0f %.0f %.0f %.0f %.2f %s %s" % (
        stage, k, fetch_b, write_b, fetch_b + write_b, particles, (fetch_b + write_b) / particles,
        "+".join(os.path.basename(x) for x in files), source_digest(files))


def read_traffic(path):
    """{stage: HBM bytes per particle} for the stages whose sources are unchanged."""
    out = {}
    if not os.path.exists(path):
        return out
    for line in open(path):
        w = line.split()
        # stage, name, kernel, fetch, write, total, particles, B/particle, sources, digest
        if len(w) == 10 and w[0] == "stage" and w[1] in STAGE_KERNELS:
            if w[9] == source_digest(STAGE_KERNELS[w[1]][1]):
                out[w[1]] = float(w[7])
    return out


def _kname(n):
    """kernel name without its argument list or template arguments"""
    n = n.replace("(anonymous namespace)::", "")
    n = n.split("(")[0]
    if n.startswith("void "):
        n = n[5:]
    return n.split("<")[0] + ("<%s>" % n.split("<", 1)[1].rsplit(">", 1)[0] if "<" in n else "")


def _csv(d, suffix):
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError("no *%s under %s" % (suffix, d))
    return hits[0]


def kernel_stats_text(d, cmd):
    rows = list(csv.DictReader(open(_csv(d, "kernel_stats.csv"))))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["# rocprofv3 --kernel-trace --stats", "# command: " + cmd,
           "%-56s %7s %10s %10s %6s" % ("kernel", "calls", "avg_us", "total_ms", "pct")]
    for r in rows:
        out.append("%-56s %7s %10.2f %10.2f %6.2f" % (
            _kname(r["Name"])[:56], r["Calls"], float(r["AverageNs"]) / 1e3,
            float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))
    return "\n".join(out)


def _per_kernel(d, skip=0):
    rows = list(csv.DictReader(open(_csv(d, "counter_collection.csv"))))
    key = "Dispatch_Id" if rows and "Dispatch_Id" in rows[0] else None
    if key:
        rows.sort(key=lambda r: int(r[key]))
    vals = defaultdict(list)
    for r in rows:
        vals[_kname(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return {k: (v[skip:] if len(v) > skip else v) for k, v in vals.items()}


def traffic_text(fetch_dir, write_dir, cal_fetch_dir, cal_write_dir, cal_bytes, bench_log, skip,
                 cmd):
    import json
    line = [l for l in open(bench_log) if l.startswith("{")][-1]
    ppl = float(json.loads(line)["config"]["mean_particles_per_step"])
    f, w = _per_kernel(fetch_dir, skip), _per_kernel(write_dir, skip)
    cf, cw = _per_kernel(cal_fetch_dir), _per_kernel(cal_write_dir)
    ck = max(cf, key=lambda k: max(cf[k]))  # the copy kernel reads the most (a fill reads nothing)
    kib = cal_bytes / 1024.0
    sf = kib / (sum(cf[ck]) / len(cf[ck]))
    sw = kib / (sum(cw[ck]) / len(cw[ck]))
    rows = {}
    for k in f:
        if k in w:
            fb = sum(f[k]) / len(f[k]) * 1024.0 * sf
            wb = sum(w[k]) / len(w[k]) * 1024.0 * sw
            rows[k] = (len(f[k]), fb, wb)
    out = ["# rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE: mean per dispatch",
           "# command: " + cmd,
           "# first %d dispatches of every kernel left out (warm-up)" % skip,
           "# calibration: %s copying %d bytes reads FETCH_SIZE x%.4f, WRITE_SIZE x%.4f of "
           "the true bytes; both scaled here" % (ck, cal_bytes, 1 / sf, 1 / sw),
           "%-48s %6s %12s %12s" % ("kernel", "disp", "fetch_MB", "write_MB")]
    for k, (n, fb, wb) in sorted(rows.items(), key=lambda kv: -(kv[1][1] + kv[1][2])):
        out.append("%-48s %6d %12.3f %12.3f" % (k[:48], n, fb / 1e6, wb / 1e6))
    out.append("# stage kernel fetch_B write_B total_B_per_launch particles_per_launch "
               "B_per_particle sources sha256")
    for s, (k, files) in STAGE_KERNELS.items():
        if k in rows:
            n, fb, wb = rows[k]
            out.append(stage_line(s, fb, wb, ppl))
    return "\n".join(out)


def copy_run(nbytes):
    import torch
    n = int(nbytes) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied %d bytes x3" % (8 * n))


def main(argv):
    if argv and argv[0] == "stats":
        print(kernel_stats_text(argv[1], " ".join(argv[2:])))
    elif argv and argv[0] == "copy":
        copy_run(int(argv[1]))
    elif argv and argv[0] == "traffic":
        print(traffic_text(argv[1], argv[2], argv[3], argv[4], int(argv[5]), argv[6],
                           int(argv[7]), " ".join(argv[8:])))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
