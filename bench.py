"""Benchmark of the r-z PIC-DSMC step on one MI355X.

Workload (default): the paper-shaped configuration -- 256 x 512 r-z cells,
5,000,000 super-particles (40 % e, 40 % Cu, 18 % Cu+, 2 % Cu2+) at W = 1,
10,300 particles injected per step, FP64 deterministic mode, seed 1.  All
inputs (initial population and the whole injection schedule) are resident
in HBM before the timed region.  A "step" is the full hot path: sort ->
collisions -> deposit -> Poisson -> field -> gather+push -> absorb ->
inject.  The metric is particle-steps per second including DSMC: the sum
over the timed steps of the particles pushed, divided by the wall time of
those steps (HIP events on the library's stream, bracketed by
synchronisation).  The stage breakdown and the roofline's kernel time come
from the same window replayed from a checkpoint taken at its start (the same
work, bit for bit), with HIP events around every stage.

Prints one JSON line.  --gpus N > 1 is not supported (one GPU only).
"""
import argparse
import json
import os
import shutil
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per particle and launch, by the real type's size F (the
# record: r, z, vr, vt, vz = 5F, species 1 B, id 4 B, key 4 B)
def algo_bytes(F):
    return {
        # read perm + record (state, species, id) at its old place, write the
        # record and its new key at the sorted place
        "push": (4 + 5 * F + 5) + (5 * F + 5 + 4),
    }


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1980)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="paper")
    ap.add_argument("--n-init", type=int, default=None)
    ap.add_argument("--poisson", choices=("direct", "spectral", "mgpcg", "learned"),
                    default="direct",
                    help="direct FP64 solve with every sum in a fixed order (bit-identical to "
                         "the oracle); the same direct solve on the FP64 matrix cores with "
                         "scan-based tridiagonal solves; FP32 multigrid CG with FP64 refinement; "
                         "or flexible CG whose first direction comes from a U-Net trained here")
    ap.add_argument("--train-samples", type=int, default=1000,
                    help="learned: (charge, potential) pairs dumped from the workload")
    ap.add_argument("--train-epochs", type=int, default=4, help="learned: training epochs")
    ap.add_argument("--precision", choices=("fp64", "fp32"), default="fp64",
                    help="FP64 deterministic, or the FP32 particle record (FP32 gather/push)")
    ap.add_argument("--ensemble", type=int, default=0,
                    help="run the batched ensemble of this many uneven replicas (FP32 records, "
                         "one HIP graph per two steps) instead of the single workload")
    ap.add_argument("--cpu-steps", type=int, default=-1,
                    help="oracle steps timed for the CPU baseline, after the same warm-up "
                         "steps as the GPU run (-1: as many as the GPU timed, capped at 40; "
                         "0: skip)")
    ap.add_argument("--form-solves", type=int, default=10,
                    help="successive node charges of the run solved by every Poisson form "
                         "(0: skip the comparison)")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles",
                                                      "hbm_traffic_paper_256x512.txt"),
                    help="rocprofv3 FETCH/WRITE summary written by "
                         "paper_2109_00214_amd.profiling traffic")
    return ap.parse_args()


def host_info():
    """CPU model and the number of cores this process may use."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "cpu_count": os.cpu_count()}


def cpu_baseline(cfg, parts, off, inj, nskip, nsteps):
    """The oracle, single-threaded, on a bounded sample of the same workload:
    nskip untimed steps from the initial state, then nsteps timed ones (the
    same window of the run as the GPU's timed steps)."""
    import oracle
    from paper_2109_00214_amd import workload as W
    o = oracle.Oracle(cfg.nr, cfg.nz, cfg.R, cfg.L, cfg.V, cfg.dt, cfg.weight, cfg.seed,
                      enable_di=cfg.enable_di)
    Z, m = W.species_table()
    o.set_species(Z, m)
    for ch, thr, dsq, sig in W.cross_section_tables():
        o.set_cross_section(ch, thr, dsq, sig)
    o.inject(parts)
    nall = nskip + nsteps
    o.schedule_injection(off[: nall + 1], {k: v[: off[nall]] for k, v in inj.items()})
    o.step(nskip)
    tot = 0
    t0 = time.perf_counter()
    for _ in range(nsteps):
        o.stage("sort")
        o.stage("collide")
        tot += o.count()
        for st in ("deposit", "poisson", "field", "push", "compact_inject", "end"):
            o.stage(st)
    dt = time.perf_counter() - t0
    out = {"value": tot / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
           "sample": "steps %d-%d of the %s workload (%d initial particles), the window the "
                     "GPU timed, single-threaded FP64 C oracle" %
                     (nskip, nskip + nsteps - 1, cfg.name, len(parts["r"])),
           "seconds": dt}
    out.update(host_info())
    return out


def train_net(a, cfg, cap, parts, precision):
    """The U-Net of the learned Poisson form, trained on the GPU on (charge,
    potential) pairs that a run of the same workload dumps (direct solves);
    none of this is inside the timed region."""
    import torch

    from paper_2109_00214_amd import pd as P
    from paper_2109_00214_amd import workload as W
    from paper_2109_00214_amd.pd import Simulation
    t1 = time.time()
    net = P.pd_unet_create(cfg.nr, cfg.nz, 4, 16, 4, a.train_samples)
    P.pd_unet_set_weights(net, W.unet_init_weights(4, 16, seed=cfg.seed))
    gen = Simulation(cfg, cap, W.cross_section_tables(), W.species_table(), precision=precision)
    gen.inject(parts)
    off_t, inj_t = W.injection_schedule(cfg, a.train_samples)
    gen.schedule_injection(off_t, inj_t)
    for _ in range(a.train_samples):
        gen.step(1)
        P.pd_unet_add_sample(net, gen.h)
    gen.close()
    t2 = time.time()
    loss = P.pd_unet_train(net, a.train_epochs, 4, 1e-3, seed=cfg.seed)
    torch.cuda.synchronize()
    learned = {"train_samples": a.train_samples, "train_epochs": a.train_epochs,
               "dump_s": round(t2 - t1, 2), "train_s": round(time.time() - t2, 2),
               "final_loss": loss, "network": "U-Net 4 levels, 16-128 channels, BF16 MFMA"}
    print("learned: %s" % learned, file=sys.stderr)
    return net, learned


def poisson_forms(cfg, charges, net):
    """Every Poisson form on the same node charges (successive steps of the
    benchmark run): device seconds per solve (HIP events around each solve),
    CG iterations and the FP64 relative residual the library measures.  The
    iterative forms start from the previous solve's potential, as in a run;
    the first solve (from the vacuum potential) is reported apart."""
    from paper_2109_00214_amd import pd as P
    from paper_2109_00214_amd import workload as W
    from paper_2109_00214_amd.pd import (PD_POISSON_DIRECT64, PD_POISSON_LEARNED,
                                         PD_POISSON_MGPCG, PD_POISSON_SPECTRAL, Simulation)
    out = {}
    for name, mode in (("direct", PD_POISSON_DIRECT64), ("spectral", PD_POISSON_SPECTRAL),
                       ("mgpcg", PD_POISSON_MGPCG), ("learned", PD_POISSON_LEARNED)):
        if name == "learned" and net is None:
            continue
        sim = Simulation(cfg, 1024, W.cross_section_tables(), W.species_table(), poisson=mode)
        if name == "learned":
            P.pd_set_unet(sim.h, net)
        rows = []
        for Q in charges:
            d0 = sim.diag()
            _, it, rel = sim.poisson(Q)
            d1 = sim.diag()
            rows.append((d1["poisson_seconds"] - d0["poisson_seconds"], int(it), float(rel),
                         d1["poisson_fallbacks"] - d0["poisson_fallbacks"]))
        warm = rows[1:] or rows
        out[name] = {"s_per_solve": sum(r[0] for r in warm) / len(warm),
                     "cg_iters_per_solve": sum(r[1] for r in warm) / len(warm),
                     "rel_res_max": max(r[2] for r in warm),
                     "fallbacks": sum(r[3] for r in rows),
                     "first_solve_s": rows[0][0], "first_solve_cg_iters": rows[0][1],
                     "solves": len(rows)}
        if name == "learned":
            P.pd_set_unet(sim.h, None)
        sim.close()
    return out


def run_ensemble(a):
    """Uneven replicas (grid, voltage, size, seed) stepped together by replaying
    one captured HIP graph of two steps; the number of worker streams of the
    capture is picked by timing each candidate (the autotuner)."""
    import torch

    from paper_2109_00214_amd import pd as P
    from paper_2109_00214_amd import workload as W
    from paper_2109_00214_amd.pd import PD_FP32_MIXED, PD_POISSON_SPECTRAL, Simulation
    cfgs = W.ensemble_configs(a.ensemble)
    cands = (1, 2, 4, 8)
    tune_steps, eager_steps = 6, 10
    nsteps = len(cands) * tune_steps + (a.warmup + 1) + (a.steps + 1) + eager_steps + 2
    torch.cuda.init()
    t0 = time.time()
    sims = []
    tables, species = W.cross_section_tables(), W.species_table()
    for k, cfg in enumerate(cfgs):
        parts = W.initial_population(cfg)
        off, inj = W.injection_schedule(cfg, nsteps)
        cap = int(1.25 * cfg.n_init + cfg.inj_cu * nsteps + 40 * cfg.inj_e + 65536)
        sim = Simulation(cfg, cap, tables, species, precision=PD_FP32_MIXED,
                         poisson=PD_POISSON_SPECTRAL)
        sim.inject(parts)
        sim.schedule_injection(off, inj)
        sims.append(sim)
        del parts
        if k % 8 == 7:
            print("replicas ready: %d of %d (%.1f s)" % (k + 1, len(cfgs), time.time() - t0),
                  file=sys.stderr, flush=True)
    hs = [s.h for s in sims]

    def pushed():
        return sum(s.diag()["particle_steps"] for s in sims)

    def timed(ens, nst):
        torch.cuda.synchronize()
        p0 = pushed()
        t = time.perf_counter()
        P.pd_ensemble_step(ens, nst)
        P.pd_ensemble_synchronize(ens)
        dt = time.perf_counter() - t
        return (pushed() - p0) / dt, dt

    tune = {}
    for ns in cands:
        ens = P.pd_ensemble_create(hs, ns)
        P.pd_ensemble_step(ens, 2)
        P.pd_ensemble_synchronize(ens)
        tune[ns] = timed(ens, tune_steps - 2)[0]
        P.pd_ensemble_destroy(ens)
    best = max(tune, key=tune.get)
    print("autotune (worker streams -> particle-steps/s): %s; using %d" % (tune, best),
          file=sys.stderr, flush=True)
    ens = P.pd_ensemble_create(hs, best)
    P.pd_ensemble_step(ens, a.warmup + (a.warmup % 2))
    P.pd_ensemble_synchronize(ens)
    ksteps = a.steps + (a.steps % 2)
    value, secs = timed(ens, ksteps)
    P.pd_ensemble_destroy(ens)
    # the same replicas stepped one launch at a time (each on its own stream)
    torch.cuda.synchronize()
    p0 = pushed()
    t = time.perf_counter()
    for _ in range(eager_steps):
        for s in sims:
            s.step(1)
    for s in sims:
        s.synchronize()
    eager = (pushed() - p0) / (time.perf_counter() - t)
    # roofline of the push over the replicas: two more steps of each with the
    # stage events on (its HIP-event time on each replica's stream)
    push_ms, units = 0.0, 0
    for s in sims:
        s.set_timing(True)
        s.timing(reset=True)
        d0 = s.diag()["particle_steps"]
        s.step(2)
        s.synchronize()
        stages, _ = s.timing()
        push_ms += stages["push"]
        units += s.diag()["particle_steps"] - d0
        s.set_timing(False)
    bpp = algo_bytes(4)["push"]
    achieved = bpp * units / (push_ms / 1e3) / 1e9
    roof = {"bound": "hbm", "kernel": "push", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "bytes_per_particle": bpp, "particles_per_launch": round(units / (2 * len(sims)))}
    n_particles = sum(c.n_init for c in cfgs)
    out = {
        "metric": "particle-steps/s incl. DSMC", "value": value, "unit": "particle-steps/s",
        "n_gpus": 1, "steps": ksteps, "warmup": a.warmup, "ms_per_step": secs * 1e3 / ksteps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "ensemble: %d replicas, 128x256 or 256x512 r-z cells, V 1-5 kV, "
                               "%d initial super-particles in all (log-uniform 0.2M-8M each), "
                               "FP32 records, matrix-core direct FP64 Poisson, one HIP graph per two steps"
                               % (len(cfgs), n_particles),
                   "replicas_256x512": sum(c.nr == 256 for c in cfgs),
                   "worker_streams": best, "autotune": {str(k): v for k, v in tune.items()},
                   "eager_particle_steps_per_s": eager},
        "roofline": roof, "cpu_baseline": None,
    }
    for s in sims:
        s.close()
    print(json.dumps(out))


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py: the step runs on one GPU only (--gpus %d requested)" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    if a.ensemble > 0:
        run_ensemble(a)
        return
    import numpy as np
    import torch

    from paper_2109_00214_amd import workload as W
    from paper_2109_00214_amd import pd as P
    from paper_2109_00214_amd.pd import (PD_FP32_MIXED, PD_FP64_DET, PD_POISSON_DIRECT64,
                                         PD_POISSON_LEARNED, PD_POISSON_MGPCG,
                                         PD_POISSON_SPECTRAL, Simulation)

    kw = {} if a.n_init is None else {"n_init": a.n_init}
    cfg = W.config(a.config, **kw)
    nsteps = a.warmup + a.steps + max(a.form_solves, 0) + 1
    t0 = time.time()
    parts = W.initial_population(cfg)
    off, inj = W.injection_schedule(cfg, nsteps)
    print("inputs ready in %.1f s: %d initial, %d scheduled" % (time.time() - t0, len(parts["r"]),
                                                                  off[-1]), file=sys.stderr)
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    cap = W.run_capacity(cfg, nsteps)
    precision = PD_FP32_MIXED if a.precision == "fp32" else PD_FP64_DET
    net, learned = None, {}
    if a.poisson == "learned":
        net, learned = train_net(a, cfg, cap, parts, precision)
    pmode = {"direct": PD_POISSON_DIRECT64, "spectral": PD_POISSON_SPECTRAL,
             "mgpcg": PD_POISSON_MGPCG, "learned": PD_POISSON_LEARNED}[a.poisson]
    sim = Simulation(cfg, cap, W.cross_section_tables(), W.species_table(), timing=True,
                     stream=stream.cuda_stream, poisson=pmode, precision=precision)
    if net is not None:
        P.pd_set_unet(sim.h, net)
    sim.inject(parts)
    sim.schedule_injection(off, inj)
    sim.set_timing(False)
    sim.step(a.warmup)
    sim.synchronize()
    # the state at the start of the timed window, to replay it with stage events
    ckpt_dir = tempfile.mkdtemp(prefix="pd_bench_")
    ckpt = os.path.join(ckpt_dir, "window_start.pd")
    sim.save(ckpt)
    d0 = sim.diag()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    sim.step(a.steps)
    e1.record(stream)
    sim.synchronize()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    d1 = sim.diag()
    pst = d1["particle_steps"] - d0["particle_steps"]
    value = pst / (ms / 1e3)
    # stage breakdown of the same window: the timed steps replayed from the
    # checkpoint (bit-identical work), each stage bracketed by HIP events on
    # the library's stream (the events cost device time, so the timed steps
    # run without them)
    sim.load(ckpt)
    shutil.rmtree(ckpt_dir, ignore_errors=True)
    sim.set_timing(True)
    sim.timing(reset=True)
    sim.step(a.steps)
    sim.synchronize()
    d2 = sim.diag()
    stages, tsteps = sim.timing()
    sim.set_timing(False)
    pst_stage = d2["particle_steps"] - d0["particle_steps"]
    if pst_stage != pst or d2["n_alive"] != d1["n_alive"]:
        raise SystemExit("bench.py: the replayed window differs from the timed one "
                         "(%d vs %d particle-steps)" % (pst_stage, pst))
    # node charges of the next steps, solved afterwards by every Poisson form
    charges = []
    for _ in range(max(a.form_solves, 0)):
        sim.step(1)
        charges.append(sim.field()["Q"].copy())
    per_step = {k: v / max(tsteps, 1) for k, v in stages.items()}
    print("stage ms/step: " + ", ".join("%s %.4f" % kv for kv in per_step.items()), file=sys.stderr)
    # roofline of the dominant single-kernel stage
    ALGO_BYTES = algo_bytes(4 if a.precision == "fp32" else 8)
    cand = {k: per_step[k] for k in ALGO_BYTES}
    dom = max(cand, key=cand.get)
    units = pst_stage / max(tsteps, 1)
    achieved = ALGO_BYTES[dom] * units / (per_step[dom] / 1e3) / 1e9
    # HBM bytes per launch: bytes per particle from the counters (taken on
    # this workload and on the kernel as it is now) times particles per launch
    from paper_2109_00214_amd.profiling import read_traffic
    bpp = read_traffic(a.traffic).get(dom) if (cfg.name == "paper" and a.n_init is None and
                                                a.precision == "fp64") else None
    traffic = round(bpp * units) if bpp is not None else None
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "bytes_per_particle": ALGO_BYTES[dom], "particles_per_launch": round(units)}
    out = {
        "metric": "particle-steps/s incl. DSMC",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if a.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "%s: %dx%d r-z cells, %d initial super-particles, W=%g, "
                               "%d injected/step, %s" %
                               (cfg.name, cfg.nr, cfg.nz, cfg.n_init, cfg.weight,
                                cfg.inj_e + cfg.inj_cu,
                                "FP32 record/gather/push, FP64 collisions" if a.precision == "fp32"
                                else "FP64 deterministic"),
                   "poisson": {"direct": "direct FP64 (sine transform + tridiagonal), "
                                         "fixed summation order",
                               "spectral": "direct FP64, transforms on the FP64 matrix cores, "
                                           "tridiagonal solves as wave scans",
                               "mgpcg": "FP32 multigrid-preconditioned CG, FP64 refinement, "
                                        "rtol 1e-8",
                               "learned": "FP32 flexible CG, first direction from the U-Net, "
                                          "then multigrid; FP64 refinement, rtol 1e-8"}[a.poisson],
                   "learned": learned or None,
                   "poisson_s_per_step": per_step["poisson"] / 1e3,
                   "poisson_rel_res_final": d1["poisson_rel_res"],
                   "poisson_cg_iters_per_step": (d1["poisson_iters"] - d0["poisson_iters"]) / a.steps,
                   "poisson_refinements_per_step":
                       (d1["poisson_refinements"] - d0["poisson_refinements"]) / a.steps,
                   "poisson_fallbacks": d1["poisson_fallbacks"],
                   "poisson_forms": None,
                   "collision_events": int(sum(d1["events"]) - sum(d0["events"])),
                   "collision_conflicts": int(d1["conflicts"] - d0["conflicts"]),
                   "mean_particles_per_step": round(units),
                   "final_particles": int(d1["n_alive"])},
        "roofline": roof,
        "stages_ms_per_step": {k: round(v, 5) for k, v in per_step.items()},
        "cpu_baseline": None,
    }
    ev = out["config"]["collision_events"]
    out["config"]["conflicts_per_event"] = (out["config"]["collision_conflicts"] / ev) if ev else None
    sim.close()
    if charges and net is None:
        net, learned = train_net(a, cfg, cap, parts, precision)
        out["config"]["learned"] = learned
    if charges:
        out["config"]["poisson_forms"] = poisson_forms(cfg, charges, net)
        print("poisson forms: %s" % json.dumps(out["config"]["poisson_forms"]), file=sys.stderr)
    if net is not None:
        P.pd_unet_destroy(net)
    ncpu = min(a.steps, 40) if a.cpu_steps < 0 else a.cpu_steps
    if ncpu > 0:
        out["cpu_baseline"] = cpu_baseline(cfg, parts, off, inj, a.warmup, ncpu)
    del np
    print(json.dumps(out))


if __name__ == "__main__":
    main()
