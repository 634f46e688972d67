"""GPU parity: the HIP library (through the C-ABI) against the CPU oracle on
the same seeded inputs.  FP64 deterministic mode: every particle value,
key, id, node charge, potential and field value and every integer count
must be bit-identical (kinetic-energy sums, whose summation order is free,
to 1e-12 relative)."""
import numpy as np
import pytest

from gpu_common import assert_same_state, gpu_sim, log, pair
from paper_2109_00214_amd import workload as W

pytestmark = pytest.mark.gpu


def _one(sp, r, z, vr, vt, vz):
    return {"r": np.array([r]), "z": np.array([z]), "vr": np.array([vr]), "vt": np.array([vt]),
            "vz": np.array([vz]), "sp": np.array([sp], np.uint8)}


def test_single_electron_uniform_field():
    log("case: single electron, vacuum field, tiny grid")
    cfg = W.config("tiny")
    a = (-W.QE) * (-cfg.V / cfg.L) / W.ME
    p = _one(W.E, 0.3e-6, 0.05e-6, 0.0, 0.0, -a * cfg.dt / 2)
    g, o = pair(cfg, parts=p, capacity=64, deposit_off=True, collisions_off=True, sched=False)
    for s in range(1, 15):
        g.step(1)
        o.step(1)
        assert_same_state(g, o, "step %d" % s)


def test_empty_domain_steps():
    log("case: empty domain")
    cfg = W.config("tiny")
    g = gpu_sim(cfg, 1024)
    g.step(3)
    d = g.diag()
    assert d["n_alive"] == 0 and d["step"] == 3 and d["events"].sum() == 0
    f = g.field()
    j = np.arange(cfg.nz + 1)
    assert np.array_equal(f["phi"][:, 0], (-cfg.V) + cfg.V * (j / cfg.nz))


@pytest.mark.parametrize("n", [1, 63, 4095, 4097, 12289])
def test_ragged_sizes_short_run(n):
    log("case: ragged population n=%d" % n)
    cfg = W.config("tiny", n_init=n)
    g, o = pair(cfg, n_init=n, steps=4)
    for s in range(1, 5):
        g.step(1)
        o.step(1)
        assert_same_state(g, o, "n=%d step %d" % (n, s))


@pytest.mark.parametrize("n", [6000, 60000])
def test_sparse_keys_paper_grid(n):
    """The 256 x 512 grid with few particles: most cells are empty (two whole
    species among them), so the cell offsets come from long runs of empty
    cells as well as from dense stretches of the sorted keys."""
    log("case: sparse keys, 256x512 grid, n=%d" % n)
    cfg = W.config("tiny", nr=256, nz=512, n_init=n)
    g, o = pair(cfg, n_init=n, steps=3)
    for s in range(1, 4):
        g.step(1)
        o.step(1)
        assert_same_state(g, o, "sparse n=%d step %d" % (n, s))


@pytest.mark.parametrize("n", [300_000, 1_200_000])
def test_many_movers_long_radix_tiles(n):
    """Populations whose first sorts have every particle (then every
    electron) moving: beyond 2^18 and 2^20 movers the mover radix passes use
    tiles of 2048 and 4096 keys, placed without the LDS reorder of the short
    tiles; the sort order and the whole state stay bit-identical."""
    log("case: many movers, 256x512 grid, n=%d" % n)
    cfg = W.config("tiny", nr=256, nz=512, n_init=n)
    g, o = pair(cfg, n_init=n, steps=3)
    for s in range(1, 4):
        g.step(1)
        o.step(1)
        assert_same_state(g, o, "many movers n=%d step %d" % (n, s))


def test_all_stayers_no_movers():
    """Neutral atoms at rest, no collisions, no injection: after the first
    sort nothing changes cell, so the sort has no movers at all (empty radix
    passes, every position a stayer) and the offsets come from the old ones
    alone."""
    log("case: all stayers")
    cfg = W.config("tiny")
    rng = np.random.default_rng(3)
    n = 5000
    p = {"r": rng.uniform(0.0, 0.99 * cfg.R, n), "z": rng.uniform(0.01 * cfg.L, 0.99 * cfg.L, n),
         "vr": np.zeros(n), "vt": np.zeros(n), "vz": np.zeros(n),
         "sp": np.full(n, W.CU, np.uint8)}
    g, o = pair(cfg, parts=p, capacity=2 * n, collisions_off=True, sched=False)
    for s in range(1, 5):
        g.step(1)
        o.step(1)
        assert_same_state(g, o, "stayers step %d" % s)


def test_tiny_config_200_steps_bit_exact():
    """32x64 cells, 50k particles, W = 100, seed 1, 200 steps."""
    cfg = W.config("tiny")
    log("case: tiny config, 200 steps")
    g, o = pair(cfg, steps=cfg.steps)
    done = 0
    for target in (1, 2, 5, 20, 60, 120, 200):
        g.step(target - done)
        o.step(target - done)
        done = target
        p = assert_same_state(g, o, "step %d" % done)
        log("  step %d ok: %d particles" % (done, len(p["r"])))
    d = g.diag()
    assert d["events"][W.DI] > 0 and d["events"][W.SI2] > 0
    assert d["particle_steps"] > 200 * 30000


def _chain_population(cfg, n_base, n_per_species, seed):
    """The workload's population plus Cu2+ of every label and Cu3+ spread
    over the volume with thermal velocities (targets of the chain)."""
    parts = W.initial_population(cfg, n=n_base)
    rng = np.random.default_rng(seed)
    extra = [parts]
    for sp in (W.CU2_STEP, W.CU2_DOUBLE, W.CU2_INIT, W.CU3):
        n = n_per_species
        extra.append({"r": cfg.R * np.sqrt(rng.random(n)) * 0.999,
                      "z": cfg.L * (0.02 + 0.96 * rng.random(n)),
                      "vr": rng.normal(0.0, 600.0, n), "vt": rng.normal(0.0, 600.0, n),
                      "vz": rng.normal(0.0, 600.0, n), "sp": np.full(n, sp, np.uint8)})
    return {k: np.concatenate([e[k] for e in extra]) for k in parts}


def test_chain_to_cu4_dense_bit_exact():
    """All six channels firing (constant cross sections with the channel
    thresholds, dense Cu2+ of every label and Cu3+): Cu3+ and Cu4+ are made
    and the whole state, Eq. 21 included, stays bit-identical."""
    log("case: step-wise chain to Cu4+, dense")
    cfg = W.config("tiny", nr=16, nz=32, weight=1e6)
    tables = W.constant_tables([2e-19] * W.NCHANNELS, thresholds=list(W.THRESHOLDS_EV), n=4096)
    parts = _chain_population(cfg, 20000, 3000, 11)
    g, o = pair(cfg, parts=parts, steps=12, tables=tables)
    for s in range(1, 13):
        g.step(1)
        o.step(1)
        assert_same_state(g, o, "chain dense step %d" % s)
    d = g.diag()
    log("  events per channel %s, Cu3+ %d, Cu4+ %d, gamma %.4f, qbar %.4f" %
        (list(d["events"]), d["count"][W.CU3], d["count"][W.CU4], d["gamma"], d["qbar"]))
    assert np.all(np.asarray(d["events"]) > 0)
    assert d["count"][W.CU4] + np.asarray(d["absorbed"])[:, W.CU4].sum() > 0


def test_chain_tiny_config_200_steps_bit_exact():
    """The tiny configuration with the Lotz tables of the whole chain."""
    log("case: tiny config with the chain to Cu4+, 200 steps")
    cfg = W.config("tiny")
    tables = W.cross_section_tables(chain=True)
    g, o = pair(cfg, parts=_chain_population(cfg, cfg.n_init, 1000, 12), steps=cfg.steps,
                tables=tables)
    done = 0
    for target in (1, 7, 50, 200):
        g.step(target - done)
        o.step(target - done)
        done = target
        assert_same_state(g, o, "chain step %d" % done)
    d = g.diag()
    log("  events per channel %s" % list(d["events"]))
    assert d["events"][W.SI3] > 0


@pytest.mark.parametrize("every", [1, 3])
def test_heavy_collisions_bit_exact(every):
    """Cu+ + Cu charge exchange and Cu + Cu elastic collisions beside the
    electron-impact channels (constant cross sections, dense heavy gas with
    drifting atoms and ions), with heavy steps every step or every third:
    every claim, label swap, scattered velocity and node charge identical."""
    log("case: heavy-projectile collisions, heavy step every %d" % every)
    cfg = W.config("tiny", nr=16, nz=32, weight=1e5)
    sig = [3e-19, 2e-19, 1e-19, 2e-19, 0.0, 0.0, 5e-18, 3e-18]
    tables = W.constant_tables(sig, thresholds=list(W.THRESHOLDS_EV), n=4096)
    parts = W.initial_population(cfg, n=30000)
    heavy = parts["sp"] != W.E
    rng = np.random.default_rng(21)
    parts["vz"] = np.where(heavy, parts["vz"] + rng.normal(0.0, 2e4, heavy.size), parts["vz"])
    g, o = pair(cfg, parts=parts, steps=15, tables=tables)
    if every > 1:
        g.set_heavy_subcycle(every)
        o.set_heavy_subcycle(every)
    for s in range(1, 16):
        g.step(1)
        o.step(1)
        assert_same_state(g, o, "heavy every %d step %d" % (every, s))
    d = g.diag()
    log("  events per channel %s, conflicts %d" % (list(d["events"]), d["conflicts"]))
    assert d["events"][W.CEX] > 100 and d["events"][W.NN] > 100


def test_all_channels_tiny_config_200_steps_bit_exact():
    """The tiny configuration with every channel's table (the chain to Cu4+,
    the heavy projectiles' stand-ins, the Coulomb channels) and the paper's
    heavy step of ten electron steps."""
    log("case: tiny config, all channels, heavy step 10, 200 steps")
    cfg = W.config("tiny")
    tables = W.cross_section_tables(chain=True, heavy=True, coulomb=True)
    g, o = pair(cfg, parts=_chain_population(cfg, cfg.n_init, 1000, 13), steps=cfg.steps,
                tables=tables)
    g.set_heavy_subcycle(10)
    o.set_heavy_subcycle(10)
    done = 0
    for target in (1, 11, 60, 200):
        g.step(target - done)
        o.step(target - done)
        done = target
        assert_same_state(g, o, "all channels step %d" % done)
    d = g.diag()
    log("  events per channel %s" % list(d["events"]))
    assert d["events"][W.CEX] > 0 and d["events"][W.NN] > 0
    assert d["events"][W.CEI] > 0 and d["events"][W.CEE] > 0


def test_coulomb_collisions_bit_exact():
    """Electron-Cu+ and electron-electron Coulomb channels beside the
    electron-impact ones on a dense population: electrons are targets too,
    so every electron event claims its projectile; the whole state stays
    bit-identical."""
    log("case: Coulomb collisions, dense")
    cfg = W.config("tiny", nr=16, nz=32, weight=1e4)
    tables = W.cross_section_tables(coulomb=True)
    g, o = pair(cfg, n_init=40000, steps=10, tables=tables)
    for s in range(1, 11):
        g.step(1)
        o.step(1)
        assert_same_state(g, o, "coulomb step %d" % s)
    d = g.diag()
    log("  events per channel %s, conflicts %d" % (list(d["events"]), d["conflicts"]))
    assert d["events"][W.CEI] > 100 and d["events"][W.CEE] > 100


def test_di_disabled_and_seed_dependence():
    log("case: DI off, seed 7")
    cfg = W.config("tiny", seed=7, enable_di=False)
    g, o = pair(cfg, steps=30)
    g.step(30)
    o.step(30)
    assert_same_state(g, o, "no-DI step 30")
    assert g.diag()["events"][W.DI] == 0


def test_dense_collisions_many_conflicts():
    """Few targets per cell and many electrons: most trials collide and many
    lose their target; ids and slots of new electrons must still match."""
    log("case: dense constant-sigma collisions")
    cfg = W.config("tiny", nr=8, nz=16, weight=1e6, V=500.0)
    tables = W.constant_tables((3e-19, 2e-19, 1e-19, 2e-19), thresholds=(0, 7.73, 28.0, 20.29),
                               n=2048)
    g, o = pair(cfg, n_init=20000, steps=10, tables=tables)
    for s in range(1, 11):
        g.step(1)
        o.step(1)
        assert_same_state(g, o, "dense step %d" % s)
    d = g.diag()
    assert d["conflicts"] > 100 and d["events"][:4].min() > 10


def test_gpu_runs_are_deterministic():
    log("case: determinism")
    cfg = W.config("tiny")
    runs = []
    for _ in range(2):
        g = gpu_sim(cfg, 200_000)
        g.inject(W.initial_population(cfg))
        off, inj = W.injection_schedule(cfg, 40)
        g.schedule_injection(off, inj)
        g.step(40)
        runs.append(g.particles())
        g.close()
    for k in runs[0]:
        assert np.array_equal(runs[0][k], runs[1][k]), k


def test_stage_timing_switch():
    """Stage events only for the steps run with timing on; the result of the
    steps does not depend on it."""
    log("case: stage timing switched off and on")
    cfg = W.config("tiny")
    parts = W.initial_population(cfg)
    off, inj = W.injection_schedule(cfg, 12)
    g = gpu_sim(cfg, 200_000, timing=True)
    g.inject(parts)
    g.schedule_injection(off, inj)
    g.step(3)
    st, n = g.timing(reset=True)
    assert n == 3 and st["permute"] == 0.0 and min(st.values()) >= 0.0
    assert st["radix"] > 0 and st["push"] > 0
    g.set_timing(False)
    g.step(5)
    st, n = g.timing()
    assert n == 0 and max(st.values()) == 0.0
    g.set_timing(True)
    g.step(4)
    st, n = g.timing()
    assert n == 4 and st["push"] > 0
    ref = gpu_sim(cfg, 200_000)
    ref.inject(parts)
    ref.schedule_injection(off, inj)
    ref.step(12)
    a, b = g.particles(), ref.particles()
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    g.close()
    ref.close()


def test_errors_leave_state_unchanged():
    from paper_2109_00214_amd.pd import PdError, PD_EINVAL, PD_ECAPACITY
    log("case: error paths")
    cfg = W.config("tiny")
    g = gpu_sim(cfg, 100)
    p = _one(W.E, 0.1e-6, 0.1e-6, 0.0, 0.0, 0.0)
    bad = dict(p)
    bad["vz"] = np.array([np.nan])
    with pytest.raises(PdError) as e:
        g.inject(bad)
    assert e.value.status == PD_EINVAL
    far = dict(p)
    far["z"] = np.array([cfg.L])
    with pytest.raises(PdError):
        g.inject(far)
    assert g.count() == 0
    many = {k: np.repeat(v, 101) for k, v in p.items()}
    with pytest.raises(PdError) as e:
        g.inject(many)
    assert e.value.status == PD_ECAPACITY
    assert g.count() == 0
    g.inject(p)
    assert g.count() == 1


def test_capacity_overflow_on_device_is_reported():
    """Injection beyond capacity inside pd_step: the device sets the error
    flag, the kernels write nothing out of bounds, and the next
    synchronising call reports PD_ECAPACITY."""
    from paper_2109_00214_amd.pd import PdError, PD_ECAPACITY
    log("case: device capacity overflow")
    cfg = W.config("tiny", inj_e=50, inj_cu=0)
    g = gpu_sim(cfg, 120, collisions_off=True)
    off, inj = W.injection_schedule(cfg, 5)
    g.schedule_injection(off, inj)
    g.step(5)
    with pytest.raises(PdError) as e:
        g.synchronize()
    assert e.value.status == PD_ECAPACITY


def test_created_electrons_beyond_capacity_are_reported():
    """Ionizations that would create more electrons than the capacity holds:
    the collision launch decides this in every block from the same chunk
    sums, creates nothing, flags the error, and the next synchronising call
    reports PD_ECAPACITY."""
    from paper_2109_00214_amd.pd import PdError, PD_ECAPACITY
    log("case: created electrons beyond capacity")
    cfg = W.config("tiny", nr=8, nz=16, weight=1e6, V=500.0, inj_e=0, inj_cu=0)
    tables = W.constant_tables((3e-19, 2e-19, 1e-19, 2e-19), thresholds=(0, 7.73, 28.0, 20.29),
                               n=2048)
    parts = W.initial_population(cfg, n=20000)
    n = len(parts["r"])
    g = gpu_sim(cfg, n + 8, tables)
    g.inject(parts)
    g.step(3)
    with pytest.raises(PdError) as e:
        g.synchronize()
    assert e.value.status == PD_ECAPACITY



@pytest.mark.parametrize("every", [10, 3])
def test_heavy_subcycle_bit_exact(every):
    """Heavy subcycling (the heavy species advance every K steps with the step
    K dt): the 32x64 workload for 200 steps, every state bit-identical to the
    oracle's with the same K, checked on heavy and on ordinary steps."""
    log("case: heavy subcycling K=%d, tiny config, 200 steps" % every)
    cfg = W.config("tiny")
    g, o = pair(cfg, steps=cfg.steps)
    g.set_heavy_subcycle(every)
    o.set_heavy_subcycle(every)
    done = 0
    for target in (1, 2, every, every + 1, 2 * every + 1, 60, 200):
        g.step(target - done)
        o.step(target - done)
        done = target
        assert_same_state(g, o, "K=%d step %d" % (every, done))
    d = g.diag()
    assert d["events"][W.DI] > 0
