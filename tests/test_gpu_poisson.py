"""GPU checks of the Poisson solvers through the C-ABI (pd_poisson): the
direct FP64 solve is bit-identical to the oracle's; the FP32 multigrid CG
with FP64 refinement reaches the relative residual 1e-8 as the oracle
measures it, on charges deposited by the oracle from seeded populations."""
import numpy as np
import pytest

from conftest import make_oracle
from gpu_common import gpu_sim, log
from paper_2109_00214_amd import workload as W
from paper_2109_00214_amd.pd import PD_POISSON_DIRECT64, PD_POISSON_MGPCG

pytestmark = pytest.mark.gpu

RTOL = 1e-8


def _charge(cfg, n):
    """Oracle deposit of a seeded population: node charge and the oracle."""
    o = make_oracle(cfg, collisions_off=True)
    if n:
        o.inject(W.initial_population(cfg, n=n))
    for st in ("sort", "collide", "deposit"):
        o.stage(st)
    return o, o.field()["Q"].copy()


def _direct(o):
    o.stage("poisson")
    return o.field()["phi"].copy()


@pytest.mark.parametrize("grid,n", [((32, 64), 50_000), ((256, 512), 300_000), ((30, 50), 20_000)])
def test_mgpcg_reaches_rtol(grid, n):
    nr, nz = grid
    log("case: MG-PCG, grid %dx%d, %d particles deposited" % (nr, nz, n))
    cfg = W.config("paper" if nr >= 256 else "tiny", nr=nr, nz=nz)
    o, Q = _charge(cfg, n)
    g = gpu_sim(cfg, 1024, poisson=PD_POISSON_MGPCG)
    phi, it, rel = g.poisson(Q)
    rn, bn = o.poisson_residual(Q, phi)
    log("  iterations %d, rel-res GPU %.3e, oracle %.3e" % (it, rel, rn / bn))
    assert rn / bn <= RTOL
    assert rel == pytest.approx(rn / bn, rel=1e-4, abs=1e-13)
    ref = _direct(o)
    err = np.max(np.abs(phi - ref)) / np.max(np.abs(ref))
    log("  max |phi - phi_direct| / max |phi_direct| = %.3e" % err)
    assert err <= 1e-6
    # electrode rows untouched
    assert np.array_equal(phi[0], ref[0]) and np.array_equal(phi[nz], ref[nz])
    # a second solve of the same charge starts converged
    phi2, it2, rel2 = g.poisson(Q)
    assert it2 == 0 and np.array_equal(phi2, phi)
    d = g.diag()
    assert d["poisson_solves"] == 2 and d["poisson_iters"] == it


def test_mgpcg_no_charge_no_voltage():
    log("case: MG-PCG, V = 0 and Q = 0")
    cfg = W.config("tiny", V=0.0)
    g = gpu_sim(cfg, 1024, poisson=PD_POISSON_MGPCG)
    Q = np.zeros((cfg.nz + 1, cfg.nr + 1), np.int64)
    phi, it, rel = g.poisson(Q)
    assert it == 0 and np.all(phi == 0.0) and rel == 0.0


def test_mgpcg_falls_back_to_direct():
    log("case: MG-PCG with an unreachable tolerance falls back to the direct solve")
    cfg = W.config("tiny")
    o, Q = _charge(cfg, 20_000)
    g = gpu_sim(cfg, 1024, poisson=PD_POISSON_MGPCG, poisson_rtol=1e-300)
    phi, it, rel = g.poisson(Q)
    ref = _direct(o)
    assert np.array_equal(phi.view(np.uint64), ref.view(np.uint64))
    assert g.diag()["poisson_fallbacks"] == 1 and it > 0


def test_direct_pd_poisson_is_bit_exact():
    log("case: direct solve through pd_poisson, 256x512")
    cfg = W.config("paper")
    o, Q = _charge(cfg, 200_000)
    g = gpu_sim(cfg, 1024, poisson=PD_POISSON_DIRECT64)
    phi, it, rel = g.poisson(Q)
    ref = _direct(o)
    assert it == 0
    assert np.array_equal(phi.view(np.uint64), ref.view(np.uint64))
    rn, bn = o.poisson_residual(Q, ref)
    # both residuals are rounding noise of the same potential
    assert rel < 1e-12 and rn / bn < 1e-12
    o.stage("field")
    fg, fo = g.field(), o.field()
    for k in ("Er", "Ez"):
        assert np.array_equal(fg[k].view(np.uint64), fo[k].view(np.uint64)), k


# grids: the paper's, the tiny one, ragged (radial nodes not a multiple of the
# eight per transform block, rows not a multiple of 64 or of the 32-row
# staging chunks), one interior row, wide radial extents (halves of 351 and
# 512 rows per tridiagonal lane, past the read-ahead runs), a tall one, and
# the smallest radial extents (one and two rows on each side of the middle)
@pytest.mark.parametrize("grid,n", [((32, 64), 50_000), ((30, 50), 20_000), ((3, 2), 2_000),
                                    ((700, 40), 100_000), ((1023, 20), 50_000),
                                    ((5, 300), 20_000), ((2, 4), 1_000), ((4, 6), 2_000)])
def test_direct_solve_bit_exact_on_ragged_grids(grid, n):
    nr, nz = grid
    log("case: fixed-order direct solve, %dx%d, %d particles" % (nr, nz, n))
    cfg = W.config("tiny", nr=nr, nz=nz)
    o, Q = _charge(cfg, n)
    g = gpu_sim(cfg, 1024, poisson=PD_POISSON_DIRECT64)
    phi, it, rel = g.poisson(Q)
    ref = _direct(o)
    assert it == 0
    bad = np.nonzero(phi.view(np.uint64) != ref.view(np.uint64))
    assert bad[0].size == 0, "first differing node (row, column): %s" % (
        [int(bad[0][0]), int(bad[1][0])],)
    o.stage("field")
    fg, fo = g.field(), o.field()
    for k in ("Er", "Ez"):
        assert np.array_equal(fg[k].view(np.uint64), fo[k].view(np.uint64)), k
    g.close()


def test_mgpcg_steps_keep_rtol():
    """The tiny workload stepped with the iterative solver: every step's
    potential meets the tolerance (checked at the end and on the way),
    nothing falls back, and the integer charge bookkeeping stays exact."""
    log("case: tiny workload, 60 steps, MG-PCG")
    cfg = W.config("tiny")
    parts = W.initial_population(cfg)
    off, inj = W.injection_schedule(cfg, 60)
    g = gpu_sim(cfg, 200_000, poisson=PD_POISSON_MGPCG)
    g.inject(parts)
    g.schedule_injection(off, inj)
    for k in range(6):
        g.step(10)
        d = g.diag()
        assert d["poisson_rel_res"] <= RTOL, (k, d["poisson_rel_res"])
    assert d["poisson_fallbacks"] == 0 and d["poisson_solves"] == 60
    assert d["charge_alive"] + d["charge_absorbed"] == d["charge_injected"]
    log("  CG iterations %d, refinements %d over 60 solves" % (d["poisson_iters"],
                                                                d["poisson_refinements"]))
    # the final potential, re-checked by the oracle for the final charge
    f = g.field()
    o = make_oracle(cfg, collisions_off=True)
    rn, bn = o.poisson_residual(f["Q"], f["phi"])
    assert rn / bn <= RTOL
