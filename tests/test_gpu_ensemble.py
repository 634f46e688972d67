"""GPU checks of ensembles: replicas of different sizes, seeds, voltages and
precisions advanced by replaying one captured HIP graph give, after every
replay (with ordinary eager calls between replays), bit-identically the state
of the same replicas stepped one by one."""
import numpy as np
import pytest

from conftest import make_oracle
from gpu_common import assert_same_state, first_diff, gpu_sim, log
from paper_2109_00214_amd import pd
from paper_2109_00214_amd import workload as W

pytestmark = pytest.mark.gpu

SPECS = [
    dict(name="tiny", seed=1, V=2900.0),
    dict(name="tiny", seed=2, V=1500.0, nr=16, nz=32, n_init=10_000),
    dict(name="tiny", seed=3, V=4000.0, nr=64, nz=128, n_init=30_000),
    dict(name="tiny", seed=4, V=2000.0, n_init=20_000, precision=pd.PD_FP32_MIXED),
]


def _replica(spec, steps):
    spec = dict(spec)
    prec = spec.pop("precision", pd.PD_FP64_DET)
    cfg = W.config(spec.pop("name"), **spec)
    g = gpu_sim(cfg, int(2 * cfg.n_init + 4 * (cfg.inj_e + cfg.inj_cu) * steps + 4096),
                precision=prec)
    g.inject(W.initial_population(cfg))
    off, inj = W.injection_schedule(cfg, steps)
    g.schedule_injection(off, inj)
    return g


def _same(a, b, where):
    d = first_diff(a.particles(), b.particles())
    assert d is None, (where, d)
    fa, fb = a.field(), b.field()
    for k in ("Q", "phi", "Er", "Ez"):
        assert np.array_equal(fa[k].view(np.uint64), fb[k].view(np.uint64)), (where, k)
    da, db = a.diag(), b.diag()
    for k in ("step", "n_alive", "next_id", "created", "conflicts", "charge_alive",
              "charge_absorbed", "charge_injected", "particle_steps", "poisson_solves"):
        assert da[k] == db[k], (where, k, da[k], db[k])
    for k in ("count", "events", "absorbed", "injected"):
        assert np.array_equal(np.asarray(da[k]), np.asarray(db[k])), (where, k)


def test_graph_replays_match_eager_steps():
    steps = 24
    refs = [_replica(s, steps) for s in SPECS]
    mems = [_replica(s, steps) for s in SPECS]
    log("case: ensemble of %d replicas (32x64, 16x32, 64x128 FP64; 32x64 FP32), graph of 2 steps"
        % len(SPECS))
    ens = pd.pd_ensemble_create([m.h for m in mems], nstreams=2)
    try:
        with pytest.raises(pd.PdError):
            mems[0].step(1)  # a member steps only through its ensemble
        for rep in range(steps // 2):
            pd.pd_ensemble_step(ens, 2)
            for r in refs:
                r.step(2)
            if rep % 3 == 2 or rep == steps // 2 - 1:
                for i, (m, r) in enumerate(zip(mems, refs)):
                    _same(m, r, "replay %d replica %d" % (rep, i))
        pd.pd_ensemble_synchronize(ens)
        assert mems[0].diag()["step"] == steps
    finally:
        pd.pd_ensemble_destroy(ens)
    # after the ensemble is gone, members step on their own again
    mems[1].step(1)
    refs[1].step(1)
    _same(mems[1], refs[1], "after the ensemble")


def test_ensemble_errors():
    log("case: ensemble argument errors")
    a = _replica(SPECS[0], 4)
    cfg = W.config("tiny")
    b = gpu_sim(cfg, 4096, poisson=pd.PD_POISSON_MGPCG)
    with pytest.raises(pd.PdError) as e:
        pd.pd_ensemble_create([a.h, b.h])
    assert e.value.status == pd.PD_EINVAL
    with pytest.raises(pd.PdError):
        pd.pd_ensemble_create([a.h, a.h])
    ens = pd.pd_ensemble_create([a.h])
    try:
        with pytest.raises(pd.PdError):
            pd.pd_ensemble_step(ens, 3)
        pd.pd_ensemble_step(ens, 0)
    finally:
        pd.pd_ensemble_destroy(ens)


def test_fp64_members_match_the_oracle():
    """Members drawn as the batched form draws its replicas (grid 128 x 256 or
    256 x 512, voltage 1-5 kV, weight 5e6 / N, their own seed), here in the FP64
    form and with the population cut to 0.2M (the smallest the batched form
    draws) so that the oracle can step beside them: after graph replays, every
    member equals, bit for bit, its own oracle stepped alongside."""
    import dataclasses
    cfgs = W.ensemble_configs(8)
    picked = [c for c in cfgs if c.nr == 128][:2] + [c for c in cfgs if c.nr == 256][:1]
    picked = [dataclasses.replace(c, n_init=200_000) for c in picked]
    steps = 8
    log("case: ensemble members against the oracle: %s" %
        [(c.nr, c.nz, round(c.V), c.n_init) for c in picked])
    mems, orcs = [], []
    for c in picked:
        parts = W.initial_population(c)
        off, inj = W.injection_schedule(c, steps)
        g = gpu_sim(c, int(1.5 * c.n_init + 4 * (c.inj_e + c.inj_cu) * steps + 65536))
        o = make_oracle(c)
        for sim in (g, o):
            sim.inject(parts)
            sim.schedule_injection(off, inj)
        mems.append(g)
        orcs.append(o)
    ens = pd.pd_ensemble_create([m.h for m in mems], nstreams=2)
    try:
        for rep in range(steps // 2):
            pd.pd_ensemble_step(ens, 2)
            pd.pd_ensemble_synchronize(ens)
            for i, (m, o) in enumerate(zip(mems, orcs)):
                o.step(2)
                assert_same_state(m, o, "replay %d member %d (%dx%d)" %
                                  (rep, i, picked[i].nr, picked[i].nz))
    finally:
        pd.pd_ensemble_destroy(ens)
    for m in mems:
        m.close()
