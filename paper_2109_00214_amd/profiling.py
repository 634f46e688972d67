"""Summaries of rocprofv3 output behind the benchmark's roofline figures.

    python -m paper_2109_00214_amd.profiling stats DIR CMD...
        kernel-trace stats (rocprofv3 --kernel-trace --stats) -> text table
    python -m paper_2109_00214_amd.profiling window DIR FIRST LAST CMD...
        the same table from the kernel trace of DIR over the steps FIRST .. LAST-1
        of the run: the launches from the first sort launch after the end of push
        launch FIRST-1 to the end of push launch LAST-1 (a step ends with its push)
    python -m paper_2109_00214_amd.profiling deposit STEPS
        the paper workload with collisions off, so that the deposit has a launch
        of its own: 5 warm-up steps, then STEPS steps; prints a JSON line whose
        config.mean_particles_per_step is the charged particles deposited per step
    python -m paper_2109_00214_amd.profiling unet REPS
        the learned solver's U-Net (4 levels, 16-128 channels) on the 256 x 512
        grid: REPS inferences of one image, for its matrix-core counters
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
    "push": ("pd::k_push<double, false>", ("csrc/k_pic.hip", "csrc/pd_internal.h")),
    "deposit": ("pd::k_deposit<double>", ("csrc/k_pic.hip", "csrc/pd_internal.h")),
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
        stage, k.replace(" ", ""), fetch_b, write_b, fetch_b + write_b, particles, (fetch_b + write_b) / particles,
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


def window_stats_text(d, first, last, cmd):
    rows = list(csv.DictReader(open(_csv(d, "kernel_trace.csv"))))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    push_end = [int(r["End_Timestamp"]) for r in rows if _kname(r["Kernel_Name"]).startswith(
        "pd::k_push")]
    if len(push_end) < last:
        raise SystemExit("only %d push launches in the trace" % len(push_end))
    # the window opens with the first sort launch after push launch first-1
    # (host-initiated copies and snapshot launches before it are not steps)
    after = push_end[first - 1] if first > 0 else -1
    lo = min(int(r["Start_Timestamp"]) for r in rows if int(r["Start_Timestamp"]) > after and
             _kname(r["Kernel_Name"]).startswith("pd::k_cls_count"))
    hi = push_end[last - 1]
    agg = defaultdict(list)
    for r in rows:
        if lo <= int(r["Start_Timestamp"]) <= hi:
            agg[_kname(r["Kernel_Name"])].append(
                int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    busy = sum(sum(v) for v in agg.values())
    nst = last - first
    out = ["# rocprofv3 --kernel-trace, steps %d-%d of the run (%d steps)" % (first, last - 1, nst),
           "# command: " + cmd,
           "# from the start of step %d's sort to the end of step %d's push: wall %.1f us per "
           "step, kernels busy %.1f us per step" % (first, last - 1, (hi - lo) / 1e3 / nst,
                                                     busy / 1e3 / nst),
           "%-56s %7s %10s %12s %6s" % ("kernel", "calls", "avg_us", "us_per_step", "pct")]
    for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        out.append("%-56s %7d %10.2f %12.2f %6.2f" % (
            k[:56], len(v), sum(v) / len(v) / 1e3, sum(v) / 1e3 / nst, 100.0 * sum(v) / busy))
    return "\n".join(out)


def deposit_run(steps):
    import json

    import torch

    from . import workload as W
    from .pd import Simulation
    cfg = W.config("paper")
    nsteps = 5 + steps
    parts = W.initial_population(cfg)
    off, inj = W.injection_schedule(cfg, nsteps)
    sim = Simulation(cfg, W.run_capacity(cfg, nsteps), W.cross_section_tables(),
                     W.species_table(), collisions_off=True)
    sim.inject(parts)
    sim.schedule_injection(off, inj)
    sim.step(5)
    Z = W.species_table()[0]
    charged = 0
    for _ in range(steps):
        # charged particles at this step's sort (the deposit's units)
        c = sim.diag()["count"]
        charged += sum(int(c[s]) for s in range(len(Z)) if Z[s] != 0)
        sim.step(1)
    sim.synchronize()
    torch.cuda.synchronize()
    sim.close()
    print(json.dumps({"config": {"workload": "paper, collisions off", "steps": steps,
                                 "mean_particles_per_step": charged / steps}}))


def unet_run(reps):
    import numpy as np

    from . import pd as P
    from . import workload as W
    net = P.pd_unet_create(256, 512, 4, 16, 1, 0)
    P.pd_unet_set_weights(net, W.unet_init_weights(4, 16, seed=1))
    _, H, Wd = P.pd_unet_info(net)
    x = np.random.default_rng(1).standard_normal((1, 2, H, Wd)).astype(np.float32)
    for _ in range(reps):
        P.pd_unet_forward(net, x)
    P.pd_unet_destroy(net)
    print("unet: %d inferences" % reps)


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
    elif argv and argv[0] == "window":
        print(window_stats_text(argv[1], int(argv[2]), int(argv[3]), " ".join(argv[4:])))
    elif argv and argv[0] == "deposit":
        deposit_run(int(argv[1]))
    elif argv and argv[0] == "unet":
        unet_run(int(argv[1]))
    elif argv and argv[0] == "copy":
        copy_run(int(argv[1]))
    elif argv and argv[0] == "traffic":
        print(traffic_text(argv[1], argv[2], argv[3], argv[4], int(argv[5]), argv[6],
                           int(argv[7]), " ".join(argv[8:])))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
