"""Pins of the oracle's boundary physics (Sec. 2.3): Fowler-Nordheim
emission from the tip with the neutral flux at a fixed ratio of the electron
flux, and the gap voltage of the external RC circuit.  The expected values
are written here from the definitions: the elementary Fowler-Nordheim law in
a uniform vacuum field, areas of annuli, the exponential decay of an RC
charge, and the charge a known number of electrons carries."""
import numpy as np
from scipy import stats

from conftest import make_oracle
from paper_2109_00214_amd import workload as W

FN_A, FN_B = 1.541434e-6, 6.830890e9  # A eV V^-2, eV^-3/2 V m^-1
PHI_W = 4.5


def _fn_current(F, area):
    return FN_A * F * F / PHI_W * np.exp(-FN_B * PHI_W ** 1.5 / F) * area


def test_emitted_count_follows_fowler_nordheim_in_a_uniform_field():
    """Vacuum field E_z = -V/L everywhere: every tip annulus sees F = beta V/L,
    the annuli inside the tip add up to pi r_tip^2, and after k steps the
    count is floor(k I dt / (e W)) up to the rounding of the carried
    fraction; the neutrals are 3 % of it."""
    cfg = W.config("tiny", nr=32, nz=64, V=2900.0, weight=1e4)
    beta, rtip = 35.0, 0.1e-6
    o = make_oracle(cfg, deposit_off=True, collisions_off=True)
    o.set_emission(beta, rtip, PHI_W, 0.03, 2000.0)
    F = beta * cfg.V / cfg.L
    I = _fn_current(F, np.pi * rtip ** 2)
    per_step = I * cfg.dt / (W.QE * cfg.weight)
    assert 10 < per_step < 1e4
    for k in (1, 2, 7, 20):
        o.step(k - (o.diag()["step"]))
        d = o.diag()
        ne, nn = d["emitted"]
        assert abs(ne - np.floor(k * per_step)) <= 1, (k, ne, k * per_step)
        assert abs(nn - np.floor(0.03 * k * per_step)) <= 1, (k, nn, 0.03 * k * per_step)


def test_emitted_positions_and_velocities():
    """Electrons start at rest on the cathode with r uniform in area over the
    tip (r^2 / r_tip^2 uniform); atoms with the normal speed of a
    flux-Maxwellian (m v^2 / (2 k T) exponential with mean 1), no
    tangential velocity."""
    cfg = W.config("tiny", nr=32, nz=64, V=2900.0, weight=100.0)
    beta, rtip, T = 35.0, 0.1e-6, 2000.0
    o = make_oracle(cfg, deposit_off=True, collisions_off=True)
    o.set_emission(beta, rtip, PHI_W, 0.5, T)
    o.stage("sort"); o.stage("collide"); o.stage("deposit"); o.stage("poisson"); o.stage("field")
    o.stage("push"); o.stage("compact_inject")
    p = o.particles()
    e, a = p["sp"] == W.E, p["sp"] == W.CU
    assert e.sum() > 1000 and a.sum() > 400
    assert np.all(p["z"] == 0.0) and np.all(p["r"] < rtip)
    assert np.all(p["vr"] == 0.0) and np.all(p["vt"] == 0.0)
    assert np.all(p["vz"][e] == 0.0)
    assert stats.kstest((p["r"][e] / rtip) ** 2, "uniform").pvalue > 1e-3
    x = W.M_CU * p["vz"][a] ** 2 / (2 * W.KB * T)
    assert stats.kstest(x, "expon").pvalue > 1e-3
    # ids continue the id sequence, electrons first
    assert np.all(np.diff(p["id"].astype(np.int64)) == 1)
    assert np.all(np.nonzero(e)[0] < np.nonzero(a)[0].min())


def test_emission_follows_the_local_field():
    """A potential whose cathode field grows with r (phi = -V + V z/L +
    c r^2 z, exact for the one-sided difference): the counts per annulus
    follow J(beta F_i) a_i (chi-square), and no field pulling the
    electrons out (F <= 0) means no emission."""
    cfg = W.config("tiny", nr=16, nz=32, V=2000.0, weight=1e3)
    beta, rtip = 35.0, 0.5e-6
    dr, dz = cfg.R / cfg.nr, cfg.L / cfg.nz
    r = np.arange(cfg.nr + 1) * dr
    z = np.arange(cfg.nz + 1) * dz
    c = 4e21  # c r_tip^2 = V/L: the field doubles across the tip
    phi = -cfg.V + cfg.V * z[:, None] / cfg.L + c * r[None, :] ** 2 * z[:, None]
    o = make_oracle(cfg, deposit_off=True, collisions_off=True)
    o.set_emission(beta, rtip, PHI_W, 0.0, 2000.0)
    o.set_potential(phi)
    o.stage("field")
    o.stage("compact_inject")
    p = o.particles()
    ring = np.floor(p["r"] / dr + 0.5).astype(int)
    lo = np.clip((np.arange(cfg.nr + 1) - 0.5) * dr, 0, rtip)
    hi = np.clip((np.arange(cfg.nr + 1) + 0.5) * dr, 0, rtip)
    area = np.pi * (hi ** 2 - lo ** 2)
    F = beta * (cfg.V / cfg.L + c * r ** 2)
    Ii = _fn_current(F, area)
    rings = np.nonzero(area > 0)[0]
    got = np.bincount(ring, minlength=cfg.nr + 1)[rings]
    exp = Ii[rings] / Ii.sum() * len(p["r"])
    assert len(p["r"]) > 2000
    assert stats.chisquare(got, exp).pvalue > 1e-3
    assert abs(len(p["r"]) - np.floor(Ii.sum() * cfg.dt / (W.QE * cfg.weight))) <= 1
    # a reversed field emits nothing
    o2 = make_oracle(cfg, deposit_off=True, collisions_off=True)
    o2.set_emission(beta, rtip, PHI_W, 0.5, 2000.0)
    o2.set_potential(-phi)
    o2.stage("field")
    o2.stage("compact_inject")
    assert o2.count() == 0


def test_circuit_relaxes_to_the_source_without_current():
    """No particles, no current: V_n = V0 + (V_init - V0)(1 - dt/(RC))^n,
    and each step's Poisson solve uses the voltage of the previous update
    (the cathode row of phi is -V)."""
    cfg = W.config("tiny", V=2000.0)
    V0, R, C = 2900.0, 1e3, 1e-12
    o = make_oracle(cfg, deposit_off=True, collisions_off=True)
    o.set_circuit(V0, R, C)
    a = 1.0 - cfg.dt / (R * C)
    v_used = cfg.V
    for n in range(1, 301):
        o.step(1)
        phi = o.field()["phi"]
        assert phi[0, 0] == -v_used
        v_used = o.diag()["V_gap"]
        expect = V0 + (cfg.V - V0) * a ** n
        assert abs(v_used - expect) <= 1e-12 * V0, (n, v_used, expect)


def test_circuit_discharge_by_absorbed_electrons():
    """Electrons absorbed at the anode take e W each from the capacitor: the
    voltage follows V <- V + (dt/C)((V0 - V)/R - I) with I = N e W / dt for
    the N electrons the previous push absorbed (counted from the absorbed
    totals), one step behind."""
    cfg = W.config("tiny", V=2900.0, weight=1e4)
    V0, R, C = 2900.0, 1e3, 1e-12
    o = make_oracle(cfg, deposit_off=True, collisions_off=True)
    rng = np.random.default_rng(3)
    n = 400
    # electrons close to the anode, moving towards it
    o.inject({"r": rng.uniform(0, 0.9 * cfg.R, n), "z": cfg.L * (1 - 1e-3 * rng.random(n)),
              "vr": np.zeros(n), "vt": np.zeros(n), "vz": rng.uniform(1e5, 1e6, n),
              "sp": np.full(n, W.E, np.uint8)})
    o.set_circuit(V0, R, C)
    V = cfg.V
    per_push = []
    tot_prev = 0
    for step in range(12):
        # the update before this step's push takes the previous push's absorptions
        I = (per_push[-1] if per_push else 0) * W.QE * cfg.weight / cfg.dt
        V = V + (cfg.dt / C) * ((V0 - V) / R - I)
        o.step(1)
        tot = int(o.diag()["absorbed"][1][W.E])
        per_push.append(tot - tot_prev)
        tot_prev = tot
        assert abs(o.diag()["V_gap"] - V) <= 1e-12 * V0, (step, o.diag()["V_gap"], V)
    assert sum(per_push) > 100
    assert o.diag()["V_gap"] < V0 - 0.01


def test_sputter_yield_threshold_and_magnitude():
    """The Cu-on-Cu yield: zero up to the threshold 6.7 U_s = 23.383 eV, the
    (1 - sqrt(E_th/E))^2.5 rise just above it (log-log slope 2.5), rising
    with energy, and of the size measured for copper self-sputtering at
    normal incidence (about 1.5-2.5 atoms per ion at 500 eV, 2-4 at 1 keV)."""
    from oracle import Oracle
    Eth = 6.7 * 3.49
    assert Oracle.sputter_yield(Eth) == 0.0 and Oracle.sputter_yield(10.0) == 0.0
    assert Oracle.sputter_yield(Eth * (1 + 1e-9)) > 0.0
    f = lambda E: 1 - np.sqrt(Eth / E)
    E1, E2 = Eth * 1.0001, Eth * 1.0002
    slope = np.log(Oracle.sputter_yield(E2) / Oracle.sputter_yield(E1)) / np.log(f(E2) / f(E1))
    assert abs(slope - 2.5) < 0.01
    ys = [Oracle.sputter_yield(E) for E in (30, 50, 100, 300, 1000, 3000)]
    assert all(b > a for a, b in zip(ys, ys[1:]))
    assert 1.5 < Oracle.sputter_yield(500.0) < 2.5
    assert 2.0 < Oracle.sputter_yield(1000.0) < 4.0


def test_sputtered_atoms_follow_the_impacts():
    """Cu+ ions driven into the cathode at known energies and radii: the
    step after the impacts, each annulus emits the whole atoms of the summed
    yields of the ions that hit nearest to its node, on the cathode, moving
    off it along z with Thompson energies E/(E + U_s)^3 (truncated at 1 keV);
    the fractions wait for the next impacts."""
    from oracle import Oracle
    cfg = W.config("tiny", V=0.0)
    dr = cfg.R / cfg.nr
    o = make_oracle(cfg, deposit_off=True, collisions_off=True)
    o.set_sputtering(True)
    rng = np.random.default_rng(7)
    n = 3000
    rings = rng.integers(0, 6, n)
    r = np.clip((rings + rng.uniform(-0.45, 0.45, n)) * dr, 0.0, None)
    E = rng.uniform(50.0, 900.0, n)
    vz = -np.sqrt(2 * E * W.QE / W.M_CU)
    z = rng.uniform(0.0, 0.5, n) * (-vz) * cfg.dt  # every ion crosses z = 0 in the first push
    o.inject({"r": r, "z": z, "vr": np.zeros(n), "vt": np.zeros(n), "vz": vz,
              "sp": np.full(n, W.CU1, np.uint8)})
    o.step(1)
    assert o.count() == 0 and o.diag()["absorbed"][0][W.CU1] == n
    o.step(1)  # the atoms of the first impacts appear at the end of this step
    p = o.particles()
    fp = np.floor(np.array([Oracle.sputter_yield(e) for e in E]) * 2.0 ** 32).astype(np.uint64)
    ring_of = np.minimum(np.floor(r / dr + 0.5).astype(int), cfg.nr)
    expect = np.zeros(cfg.nr + 1, np.int64)
    for i in range(cfg.nr + 1):
        expect[i] = int(fp[ring_of == i].sum(dtype=np.uint64)) >> 32
    got = np.bincount(np.minimum(np.floor(p["r"] / dr + 0.5).astype(int), cfg.nr),
                      minlength=cfg.nr + 1)
    assert expect.sum() > 1000
    assert np.array_equal(got, expect)
    assert o.diag()["sputtered"] == expect.sum()
    assert np.all(p["sp"] == W.CU) and np.all(p["z"] == 0.0) and np.all(p["vz"] > 0.0)
    Es = 0.5 * W.M_CU * p["vz"] ** 2 / W.QE
    Us, Emax = 3.49, 1000.0
    cdf = lambda e: (e / (e + Us)) ** 2 / (Emax / (Emax + Us)) ** 2
    assert np.all(Es <= Emax * (1 + 1e-12))
    assert stats.kstest(Es, cdf).pvalue > 1e-3
