"""GPU checks of the matrix-core form of the direct Poisson solve
(PD_POISSON_SPECTRAL: FP64 MFMA sine transforms, tridiagonal recurrences as
wave scans) against the FP64 oracle.  The solve evaluates the same equations
as the sequential direct solve in another order, so the bar is rounding:

  - potential: max |phi - phi_oracle| / max |phi_oracle| <= 1e-12, and the
    oracle's relative residual of the GPU potential <= 1e-12;
  - field: max |E - E_oracle| / max |E_oracle| <= 1e-10;
  - the tiny workload stepped 200 times: particle counts, species, ids, cell
    keys (hence the sort order) and per-channel event counts identical to
    the oracle's; positions and velocities within 1e-10 of the extent and of
    the largest speed (the tolerance the method is held to after 200 steps).
"""
import numpy as np
import pytest

from conftest import make_oracle
from gpu_common import gpu_sim, log
from paper_2109_00214_amd import workload as W
from paper_2109_00214_amd.pd import PD_POISSON_SPECTRAL

pytestmark = pytest.mark.gpu

TOL_PHI = 1e-12
TOL_E = 1e-10
TOL_STATE = 1e-10


def _charge(cfg, n):
    o = make_oracle(cfg, collisions_off=True)
    if n:
        o.inject(W.initial_population(cfg, n=n))
    for st in ("sort", "collide", "deposit"):
        o.stage(st)
    return o, o.field()["Q"].copy()


def _maxrel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# grids: the paper's, the tiny one, ragged tiles (W, nz - 1 not multiples of
# 16), one interior row, and wide ones (11 and 16 radial rows per lane)
@pytest.mark.parametrize("grid,n", [((256, 512), 300_000), ((32, 64), 50_000), ((30, 50), 20_000),
                                    ((3, 2), 2_000), ((700, 40), 100_000), ((1023, 20), 50_000)])
def test_spectral_solve_matches_oracle(grid, n):
    nr, nz = grid
    cfg = W.config("tiny", nr=nr, nz=nz)
    log("case: spectral direct solve, %dx%d, %d particles" % (nr, nz, n))
    o, Q = _charge(cfg, n)
    g = gpu_sim(cfg, 1024, poisson=PD_POISSON_SPECTRAL)
    phi, it, rel = g.poisson(Q)
    o.stage("poisson")
    o.stage("field")
    fo = o.field()
    e = _maxrel(phi, fo["phi"])
    rn, bn = o.poisson_residual(Q, phi)
    log("  potential: max rel %.2e, oracle residual %.2e, library residual %.2e" % (e, rn / bn, rel))
    assert it == 0 and e <= TOL_PHI and rn / bn <= TOL_PHI and rel <= TOL_PHI
    fg = g.field()
    for k in ("Er", "Ez"):
        ek = _maxrel(fg[k], fo[k])
        log("  %s: max rel %.2e" % (k, ek))
        assert ek <= TOL_E, k
    # the electrode rows are the vacuum values exactly
    assert np.array_equal(phi[0], fo["phi"][0]) and np.array_equal(phi[-1], fo["phi"][-1])
    g.close()


def test_spectral_no_charge_is_vacuum():
    cfg = W.config("tiny")
    o, Q = _charge(cfg, 0)
    g = gpu_sim(cfg, 1024, poisson=PD_POISSON_SPECTRAL)
    phi, _, _ = g.poisson(Q)
    o.stage("poisson")
    ref = o.field()["phi"]
    assert _maxrel(phi, ref) <= 1e-15
    g.close()


def _by_id(p):
    order = np.argsort(p["id"], kind="stable")
    return {k: v[order] for k, v in p.items()}


def test_spectral_tiny_200_steps():
    cfg = W.config("tiny")
    log("case: tiny workload, 200 steps, spectral direct solve against the oracle")
    parts = W.initial_population(cfg)
    n = len(parts["r"])
    g = gpu_sim(cfg, int(2 * n + 4 * (cfg.inj_e + cfg.inj_cu) * cfg.steps + 4096),
                poisson=PD_POISSON_SPECTRAL)
    o = make_oracle(cfg)
    g.inject(parts)
    o.inject(parts)
    off, inj = W.injection_schedule(cfg, cfg.steps)
    g.schedule_injection(off, inj)
    o.schedule_injection(off, inj)
    done = 0
    for target in (1, 20, 100, 200):
        g.step(target - done)
        o.step(target - done)
        done = target
        a, b = g.particles(), o.particles()
        assert len(a["r"]) == len(b["r"]), done
        # integer state in sorted order: identical (the sort order included)
        for k in ("sp", "id", "key"):
            assert np.array_equal(a[k], b[k]), (done, k)
        err = {}
        for k, scale in (("r", cfg.R), ("z", cfg.L)):
            err[k] = float(np.max(np.abs(a[k] - b[k]))) / scale
        vmax = max(float(np.max(np.abs(b[k]))) for k in ("vr", "vt", "vz"))
        for k in ("vr", "vt", "vz"):
            err[k] = float(np.max(np.abs(a[k] - b[k]))) / vmax
        log("  step %d: %d particles, max rel error %s" %
            (done, len(a["r"]), {k: "%.1e" % v for k, v in err.items()}))
        assert max(err.values()) <= TOL_STATE, (done, err)
    dg, do = g.diag(), o.diag()
    assert [int(x) for x in dg["events"]] == [int(x) for x in do["events"]]
    assert [int(x) for x in dg["count"]] == [int(x) for x in do["count"]]
    fg, fo = g.field(), o.field()
    assert np.array_equal(fg["Q"], fo["Q"])
    assert _maxrel(fg["phi"], fo["phi"]) <= TOL_STATE
    g.close()
