"""Shared helpers of the GPU parity tests: one seeded input set drives both
the HIP library (through the C-ABI binding) and the CPU oracle."""
import sys

import numpy as np

from conftest import make_oracle
from paper_2109_00214_amd import workload as W

FIELDS = ("r", "z", "vr", "vt", "vz", "sp", "id", "key")


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_sim(cfg, capacity, tables=None, **kw):
    from paper_2109_00214_amd.pd import Simulation
    return Simulation(cfg, capacity, tables or W.cross_section_tables(), W.species_table(), **kw)


def pair(cfg, n_init=None, steps=0, capacity=None, tables=None, parts=None, sched=True, **kw):
    """GPU simulation and oracle fed the same initial population and schedule."""
    parts = W.initial_population(cfg, n=n_init) if parts is None else parts
    n = len(parts["r"])
    if capacity is None:
        capacity = int(2 * n + 4 * (cfg.inj_e + cfg.inj_cu) * max(steps, 1) + 4096)
    g = gpu_sim(cfg, capacity, tables, **kw)
    o = make_oracle(cfg, tables=tables, **kw)
    if n:
        g.inject(parts)
        o.inject(parts)
    if sched and steps:
        off, inj = W.injection_schedule(cfg, steps)
        g.schedule_injection(off, inj)
        o.schedule_injection(off, inj)
    return g, o


def first_diff(a, b):
    """Name, index and values of the first differing particle field, or None."""
    if len(a["r"]) != len(b["r"]):
        return ("count", len(a["r"]), len(b["r"]))
    for k in FIELDS:
        x, y = a[k], b[k]
        if x.dtype.kind == "f":
            bad = np.nonzero(x.view(np.uint64) != y.view(np.uint64))[0]
        else:
            bad = np.nonzero(x != y)[0]
        if bad.size:
            i = int(bad[0])
            return (k, i, x[i], y[i], int(bad.size))
    return None


def assert_same_state(g, o, where=""):
    pg, po = g.particles(), o.particles()
    d = first_diff(pg, po)
    assert d is None, "first difference %s: %s" % (where, d)
    fg, fo = g.field(), o.field()
    assert np.array_equal(fg["Q"], fo["Q"]), where + " Q"
    for k in ("phi", "Er", "Ez"):
        assert np.array_equal(fg[k].view(np.uint64), fo[k].view(np.uint64)), where + " " + k
    dg, do = g.diag(), o.diag()
    for k in ("n_alive", "next_id", "conflicts", "created", "charge_alive", "charge_absorbed",
              "charge_injected"):
        assert dg[k] == do[k], (where, k, dg[k], do[k])
    for k in ("count", "events", "absorbed", "injected"):
        assert np.array_equal(np.asarray(dg[k]), np.asarray(do[k])), (where, k, dg[k], do[k])
    np.testing.assert_allclose(dg["ke_J"], do["ke_J"], rtol=1e-12, atol=0)
    for t in range(3):
        assert np.array_equal(g.spectrum(t), do["spectrum"][t]), (where, "spectrum", t)
    return pg
