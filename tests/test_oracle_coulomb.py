"""Pins of the oracle's Coulomb collisions (Sec. 2.3 lists them without a
model): electron-Cu+ and electron-electron elastic channels whose cross
section is the momentum-transfer cross section 4 pi lnL b90^2 of a pair of
unit charges, b90 = e^2 / (4 pi eps0 m_r g^2) the impact parameter of a
90-degree deflection, tabulated like the others in sqrt(E_rel)."""
import numpy as np
import pytest
from scipy import stats

from conftest import make_oracle
from paper_2109_00214_amd import workload as W


def test_cross_section_is_the_momentum_transfer_form():
    """The table generator against b90 written with the pair's reduced mass
    and relative speed: the table depends on E_rel = m_r g^2 / 2 only, so the
    electron-ion and electron-electron pairs share it."""
    for mr in (W.ME * W.M_CU / (W.ME + W.M_CU), W.ME / 2):
        for g in (3e5, 1e6, 5e6):
            b90 = W.QE ** 2 / (4 * np.pi * W.EPS0 * mr * g * g)
            E = 0.5 * mr * g * g / W.QE
            ref = 4 * np.pi * 10.0 * b90 * b90
            assert abs(W.coulomb_sigma(E) - ref) <= 1e-12 * ref


def _gas(cfg, groups, seed):
    rng = np.random.default_rng(seed)
    C = cfg.nr * cfg.nz
    dr, dz = cfg.R / cfg.nr, cfg.L / cfg.nz
    out = {k: [] for k in ("r", "z", "vr", "vt", "vz", "sp")}
    for sp, cnt, vz in groups:
        c = np.repeat(np.arange(C), cnt)
        out["r"].append((c % cfg.nr + 0.05 + 0.9 * rng.random(c.size)) * dr)
        out["z"].append((c // cfg.nr + 0.05 + 0.9 * rng.random(c.size)) * dz)
        out["vr"].append(np.zeros(c.size))
        out["vt"].append(np.zeros(c.size))
        out["vz"].append(np.full(c.size, vz))
        out["sp"].append(np.full(c.size, sp, np.uint8))
    return {k: np.concatenate(v) for k, v in out.items()}


def _tables(cei, cee):
    tabs = [(k, 0.0, 2.0 ** -4, np.zeros(1025)) for k in (W.EL, W.SI, W.DI, W.SI2)]
    if cei:
        tabs.append((W.CEI, 0.0, 2.0 ** -4, W.coulomb_sigma((np.arange(1025) * 2.0 ** -4) ** 2)))
    if cee:
        tabs.append((W.CEE, 0.0, 2.0 ** -4, W.coulomb_sigma((np.arange(1025) * 2.0 ** -4) ** 2)))
    return tabs


def _sigma_table(E):
    """the oracle's interpolation of the generated table at E (eV)"""
    sq = np.arange(1025) * 2.0 ** -4
    return np.interp(np.sqrt(E), sq, W.coulomb_sigma(sq ** 2))


def test_electron_ion_rate():
    """A beam at v through Cu+ at rest: passed trials = sum of
    1 - exp(-dt v n sigma(E_rel)) within 3 sigma."""
    v = 4.0e6
    n_ion, n_e = 30, 2
    mr = W.ME * W.M_CU / (W.ME + W.M_CU)
    E = 0.5 * mr * v * v / W.QE
    expect = got = 0.0
    for trial in range(10):
        cfg = W.config("tiny", nr=8, nz=16, weight=1e6, seed=10 + trial)
        o = make_oracle(cfg, tables=_tables(True, False), deposit_off=True)
        o.inject(_gas(cfg, [(W.CU1, n_ion, 0.0), (W.E, n_e, v)], trial))
        o.stage("sort")
        n = o.count()
        o.stage("collide")
        ch, tg, wn = o.collisions(n)
        got += int((ch == W.CEI + 1).sum())
        _, vc = o.node_volumes()
        i = np.arange(cfg.nr * cfg.nz) % cfg.nr
        x = cfg.dt * v * (n_ion * cfg.weight / vc[i]) * _sigma_table(E)
        expect += n_e * (-np.expm1(-x)).sum()
    assert 50 < expect
    assert abs(got - expect) < 3 * np.sqrt(expect), (got, expect)


def test_electron_electron_rate_no_self_pairs():
    """Two electron groups per cell, at rest and at v: a partner is one of the
    other N - 1 electrons, g = v across the groups, 0 within; the trial
    carries the factor 1/2 (both sides)."""
    v = 3.0e6
    nA, nB = 6, 4
    N = nA + nB
    E = 0.5 * (W.ME / 2) * v * v / W.QE
    expect = got = 0.0
    for trial in range(10):
        cfg = W.config("tiny", nr=8, nz=16, weight=1e6, seed=40 + trial)
        o = make_oracle(cfg, tables=_tables(False, True), deposit_off=True)
        o.inject(_gas(cfg, [(W.E, nA, 0.0), (W.E, nB, v)], trial))
        o.stage("sort")
        n = o.count()
        b = o.particles()
        o.stage("collide")
        ch, tg, wn = o.collisions(n)
        sel = np.nonzero(ch == W.CEE + 1)[0]
        got += sel.size
        assert np.all(tg[sel] != sel) and np.all(b["sp"][tg[sel]] == W.E)
        assert np.all(b["key"][tg[sel]] == b["key"][sel])
        _, vc = o.node_volumes()
        i = np.arange(cfg.nr * cfg.nz) % cfg.nr
        p = -np.expm1(-0.5 * cfg.dt * v * ((N - 1) * cfg.weight / vc[i]) * _sigma_table(E))
        expect += ((nA * nB / (N - 1)) * p + (nB * nA / (N - 1)) * p).sum()
    assert 50 < expect
    assert abs(got - expect) < 3 * np.sqrt(expect), (got, expect)


def test_identities_and_one_event_per_particle():
    """Both channels are elastic: each event keeps its pair's momentum and
    energy and every label; with electron-electron collisions no electron
    takes part in two events (an electron event claims its projectile too)."""
    cfg = W.config("tiny", nr=4, nz=8, weight=1e7)
    parts = _gas(cfg, [(W.CU1, 20, 0.0), (W.E, 12, 0.0)], 5)
    rng = np.random.default_rng(6)
    e = parts["sp"] == W.E
    for k in ("vr", "vt", "vz"):
        parts[k] = np.where(e, rng.normal(0.0, 2e6, e.size), rng.normal(0.0, 500.0, e.size))
    o = make_oracle(cfg, tables=_tables(True, True), deposit_off=True)
    o.inject(parts)
    o.stage("sort")
    n = o.count()
    b = o.particles()
    o.stage("collide")
    a = o.particles()
    ch, tg, wn = o.collisions(n)
    win = np.nonzero(wn)[0]
    kinds = ch[win] - 1
    assert (kinds == W.CEI).sum() > 20 and (kinds == W.CEE).sum() > 20
    who = np.concatenate([win, tg[win]])
    assert np.unique(who).size == who.size
    m = np.where(b["sp"] == W.E, W.ME, W.M_CU)
    for p in win:
        t = tg[p]
        v0 = np.array([[b[k][p], b[k][t]] for k in ("vr", "vt", "vz")])
        v1 = np.array([[a[k][p], a[k][t]] for k in ("vr", "vt", "vz")])
        mm = np.array([m[p], m[t]])
        assert np.allclose(v1 @ mm, v0 @ mm, rtol=0, atol=1e-12 * np.abs(v0 @ mm).max() + 1e-30)
        e0, e1 = (mm * (v0 ** 2).sum(axis=0)).sum(), (mm * (v1 ** 2).sum(axis=0)).sum()
        assert abs(e1 - e0) <= 1e-12 * e0
        assert a["sp"][p] == b["sp"][p] and a["sp"][t] == b["sp"][t]
    d = o.diag()
    assert int(np.sum(d["events"])) + d["conflicts"] == int((ch > 0).sum())


def test_coulomb_channels_absent_without_tables():
    cfg = W.config("tiny", n_init=20_000)
    parts = W.initial_population(cfg)
    base = W.cross_section_tables()
    zero = [(W.CEI, 0.0, 2.0 ** -4, np.zeros(1025)), (W.CEE, 0.0, 2.0 ** -4, np.zeros(1025))]
    runs = []
    for tabs in (base, base + zero):
        o = make_oracle(cfg, tables=tabs)
        o.inject(parts)
        o.step(20)
        runs.append(o.particles())
    for k in runs[0]:
        assert np.array_equal(runs[0][k], runs[1][k]), k
