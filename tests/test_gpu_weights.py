"""GPU parity of unequal weights (integer multiplicities, the rejection
reading of Sec. 2.2) against the oracle: the weighted deposit, Eq. 4's
weighted target density, the side rejection of every channel and the
multiplicities of created electrons, bit for bit; multiplicities of 1 leave
every result as without them; a checkpoint carries them."""
import numpy as np
import pytest

from conftest import make_oracle
from gpu_common import assert_same_state, gpu_sim, log
from paper_2109_00214_amd import workload as W
from paper_2109_00214_amd.pd import PdError
from test_gpu_parity import _chain_population

pytestmark = pytest.mark.gpu


def _weighted_pair(cfg, parts, mult, steps, tables=None):
    n = len(parts["r"])
    capacity = int(2 * n + 4 * (cfg.inj_e + cfg.inj_cu) * max(steps, 1) + 4096)
    g = gpu_sim(cfg, capacity, tables)
    g.set_weighted(True)
    o = make_oracle(cfg, tables=tables)
    g.inject(parts, mult)
    o.inject(parts, mult)
    if steps:
        off, inj = W.injection_schedule(cfg, steps)
        g.schedule_injection(off, inj)
        o.schedule_injection(off, inj)
    return g, o


def _check(g, o, where):
    assert_same_state(g, o, where)
    assert np.array_equal(g.weights(), o.weights()), where + " multiplicities"


def test_unit_multiplicities_change_nothing():
    """Multiplicities on, all 1: the tiny configuration stays bit-identical to
    the oracle (which then draws nothing more and weights nothing)."""
    log("case: weights on, all multiplicities 1, tiny config, 60 steps")
    cfg = W.config("tiny")
    parts = W.initial_population(cfg)
    g, o = _weighted_pair(cfg, parts, None, 60)
    done = 0
    for target in (1, 20, 60):
        g.step(target - done)
        o.step(target - done)
        done = target
        _check(g, o, "unit weights step %d" % done)
    assert np.all(g.weights() == 1)


def test_tiny_config_random_multiplicities_200_steps():
    """The tiny configuration with multiplicities 1..6 on the initial
    population (the scheduled particles stand for W): every particle, its
    multiplicity, Q, phi, E, the counters and Eq. 21 over the real numbers
    bit-identical over 200 steps."""
    log("case: tiny config, multiplicities 1..6, 200 steps")
    cfg = W.config("tiny")
    parts = W.initial_population(cfg)
    mult = np.random.default_rng(31).integers(1, 7, len(parts["r"])).astype(np.uint16)
    g, o = _weighted_pair(cfg, parts, mult, cfg.steps)
    done = 0
    for target in (1, 7, 50, 200):
        g.step(target - done)
        o.step(target - done)
        done = target
        _check(g, o, "weighted tiny step %d" % done)
    d = g.diag()
    w = g.weights()
    log("  events %s, created %d, multiplicities > 1: %d of %d" %
        (list(d["events"]), d["created"], int((w > 1).sum()), w.size))
    assert d["created"] > 0 and int((w > 1).sum()) > 1000


def test_dense_every_channel_random_multiplicities():
    """Every channel (the chain to Cu4+, charge exchange and Cu-Cu elastic on
    every step, the Coulomb channels) on a dense population with
    multiplicities 1..8: the rejection decides differently for each pair,
    created electrons take their target's multiplicity; bit-identical over
    12 steps."""
    log("case: dense, every channel, multiplicities 1..8")
    cfg = W.config("tiny", nr=16, nz=32, weight=2e5)
    sig = [2e-19] * 6 + [5e-18, 3e-18, 0.0, 0.0]
    tables = W.constant_tables(sig, thresholds=list(W.THRESHOLDS_EV), n=4096)
    tables += [t for t in W.cross_section_tables(coulomb=True) if t[0] in (W.CEI, W.CEE)]
    parts = _chain_population(cfg, 20000, 2000, 17)
    mult = np.random.default_rng(32).integers(1, 9, len(parts["r"])).astype(np.uint16)
    g, o = _weighted_pair(cfg, parts, mult, 12, tables)
    for s in range(1, 13):
        g.step(1)
        o.step(1)
        _check(g, o, "weighted dense step %d" % s)
    d = g.diag()
    log("  events per channel %s, conflicts %d, real %s" %
        (list(d["events"]), d["conflicts"], list(d["real"])))
    assert np.asarray(d["events"])[:8].min() > 10
    assert not np.array_equal(np.asarray(d["real"]), np.asarray(d["count"]))


def test_resume_with_multiplicities_is_bit_exact(tmp_path):
    """40 steps equal 20 steps + pd_save + pd_load into a fresh context +
    20 steps, multiplicities included."""
    log("case: weighted checkpoint resume")
    cfg = W.config("tiny")
    parts = W.initial_population(cfg)
    mult = np.random.default_rng(33).integers(1, 5, len(parts["r"])).astype(np.uint16)
    g, o = _weighted_pair(cfg, parts, mult, 40)
    g.step(20)
    path = str(tmp_path / "w.pd")
    g.save(path)
    h = gpu_sim(cfg, int(2 * len(parts["r"]) + 4 * (cfg.inj_e + cfg.inj_cu) * 40 + 4096))
    h.load(path)
    g.step(20)
    h.step(20)
    o.step(40)
    _check(g, o, "weighted straight 40")
    _check(h, o, "weighted resumed 20 + 20")


def test_multiplicity_errors():
    cfg = W.config("tiny")
    parts = W.initial_population(cfg, n=100)
    g = gpu_sim(cfg, 10000)
    with pytest.raises(PdError):  # not enabled
        g.inject(parts, np.ones(100, np.uint16))
    g.set_weighted(True)
    bad = np.ones(100, np.uint16)
    bad[7] = 0
    with pytest.raises(PdError):
        g.inject(parts, bad)
    assert g.count() == 0
    with pytest.raises(PdError):  # no circuit with multiplicities
        g.set_circuit(2900.0, 1e3, 1e-12)
    with pytest.raises(PdError):  # cannot be turned off
        g.set_weighted(False)
    h = gpu_sim(cfg, 10000)
    h.set_circuit(2900.0, 1e3, 1e-12)
    with pytest.raises(PdError):
        h.set_weighted(True)
    f = gpu_sim(cfg, 10000, precision=1)
    with pytest.raises(PdError):  # FP64 record only
        f.set_weighted(True)
