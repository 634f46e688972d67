"""Pins of the oracle's gather + leapfrog push (paper Sec. 2.1, Newton's law in
2D3V r-z geometry) against closed-form trajectories."""
import numpy as np

from conftest import make_oracle
from paper_2109_00214_amd import workload as W


def _one(sp, r, z, vr, vt, vz):
    return {"r": np.array([r]), "z": np.array([z]), "vr": np.array([vr]),
            "vt": np.array([vt]), "vz": np.array([vz]), "sp": np.array([sp], np.uint8)}


def test_uniform_field_trajectory_electron():
    """Electron in the vacuum field E_z = -V/L: leapfrog is exact for
    constant acceleration when v(-1/2) = v0 - a dt/2; r stays fixed."""
    cfg = W.config("tiny")
    o = make_oracle(cfg, deposit_off=True, collisions_off=True)
    a = (-W.QE) * (-cfg.V / cfg.L) / W.ME
    r0, z0 = 0.3e-6, 0.05e-6
    o.inject(_one(W.E, r0, z0, 0.0, 0.0, -a * cfg.dt / 2))
    for n in range(1, 200):
        o.step(1)
        if o.count() == 0:
            break
        p = o.particles()
        t = n * cfg.dt
        assert p["r"][0] == r0
        assert p["vr"][0] == 0.0 and p["vt"][0] == 0.0
        assert abs(p["z"][0] - (z0 + 0.5 * a * t * t)) <= 1e-12 * cfg.L
        assert abs(p["vz"][0] - a * (n - 0.5) * cfg.dt) <= 1e-11 * abs(a * n * cfg.dt)
    assert o.count() == 0
    d = o.diag()
    assert d["absorbed"][1][W.E] == 1  # reached the anode
    assert (z0 + 0.5 * a * (n * cfg.dt) ** 2) >= cfg.L > (z0 + 0.5 * a * ((n - 1) * cfg.dt) ** 2)


def test_uniform_field_ion_goes_to_cathode():
    cfg = W.config("tiny")
    o = make_oracle(cfg, deposit_off=True, collisions_off=True)
    a = (2 * W.QE) * (-cfg.V / cfg.L) / W.M_CU
    z0 = 1.5e-6
    o.inject(_one(W.CU2_INIT, 0.2e-6, z0, 0.0, 0.0, -a * cfg.dt / 2))
    n = 0
    while o.count():
        o.step(1)
        n += 1
        if o.count():
            p = o.particles()
            assert abs(p["z"][0] - (z0 + 0.5 * a * (n * cfg.dt) ** 2)) <= 1e-12 * cfg.L
    assert o.diag()["absorbed"][0][W.CU2_INIT] == 1


def test_free_streaming_cylindrical():
    """Field-free motion: r(t) = |(r0 + vr t, vt t)|, z = z0 + vz t; r*v_theta
    (angular momentum per mass) is invariant; crossing near the axis."""
    cfg = W.config("tiny", V=0.0)
    o = make_oracle(cfg, deposit_off=True, collisions_off=True)
    r0, z0, vr, vt, vz = 0.4e-6, 0.5e-6, -3.0e5, 2.0e4, 1.0e5
    o.inject(_one(W.CU, r0, z0, vr, vt, vz))
    L0 = r0 * vt
    for n in range(1, 250):
        o.step(1)
        p = o.particles()
        t = n * cfg.dt
        r_ex = np.hypot(r0 + vr * t, vt * t)
        assert abs(p["r"][0] - r_ex) <= 1e-12 * r0
        assert abs(p["z"][0] - (z0 + vz * t)) <= 1e-12 * cfg.L
        assert abs(p["r"][0] * p["vt"][0] - L0) <= 1e-10 * abs(L0)
        speed = np.sqrt(p["vr"][0] ** 2 + p["vt"][0] ** 2)
        assert abs(speed - np.hypot(vr, vt)) <= 1e-12 * np.hypot(vr, vt)


def test_field_free_has_no_force_on_neutrals_in_field():
    """Neutrals (Z = 0) move in a straight line even in the gap field."""
    cfg = W.config("tiny")
    o = make_oracle(cfg, deposit_off=True, collisions_off=True)
    o.inject(_one(W.CU, 0.1e-6, 0.1e-6, 0.0, 0.0, 2.0e4))
    for n in range(1, 50):
        o.step(1)
    p = o.particles()
    assert abs(p["z"][0] - (0.1e-6 + 2.0e4 * 49 * cfg.dt)) < 1e-20
    assert p["vz"][0] == 2.0e4


def test_heavy_subcycle_uniform_field_ion():
    """Heavy subcycling with K = 10 (Sec. 2.3: the heavy particles' step is ten
    times the electrons'): the ion moves only on the steps whose counter is a
    multiple of K, each time by the leapfrog step K dt, which is exact for a
    constant acceleration when v(-1/2) = v0 - a K dt / 2; r stays fixed; in
    between, the position does not change at all."""
    cfg = W.config("tiny")
    K = 10
    o = make_oracle(cfg, deposit_off=True, collisions_off=True)
    o.set_heavy_subcycle(K)
    dth = K * cfg.dt
    a = (2 * W.QE) * (-cfg.V / cfg.L) / W.M_CU
    z0, r0 = 1.5e-6, 0.2e-6
    o.inject(_one(W.CU2_INIT, r0, z0, 0.0, 0.0, -a * dth / 2))
    m = 0
    z_prev = z0
    for n in range(1, 5000):
        o.step(1)
        if o.count() == 0:
            break
        p = o.particles()
        if (n - 1) % K == 0:
            m += 1
            assert abs(p["z"][0] - (z0 + 0.5 * a * (m * dth) ** 2)) <= 1e-12 * cfg.L, n
            assert abs(p["vz"][0] - a * (m - 0.5) * dth) <= 1e-11 * abs(a * m * dth), n
        else:
            assert p["z"][0] == z_prev, n
        assert p["r"][0] == r0 and p["vr"][0] == 0.0 and p["vt"][0] == 0.0
        z_prev = p["z"][0]
    assert o.count() == 0 and (n - 1) % K == 0  # absorbed on a heavy step
    assert o.diag()["absorbed"][0][W.CU2_INIT] == 1
    # the absorbing heavy step is the one whose exact position crosses the
    # cathode (to the rounding of the exact formula)
    m += 1
    assert (z0 + 0.5 * a * (m * dth) ** 2) < 1e-12 * cfg.L
    assert (z0 + 0.5 * a * ((m - 1) * dth) ** 2) > 0.0


def test_heavy_subcycle_leaves_electrons_alone():
    """In the vacuum field an electron's trajectory does not depend on the
    heavy step (bit for bit), and with K = 1 nothing changes at all."""
    cfg = W.config("tiny")
    runs = {}
    for K in (None, 1, 10):
        o = make_oracle(cfg, deposit_off=True, collisions_off=True)
        if K is not None:
            o.set_heavy_subcycle(K)
        o.inject(_one(W.E, 0.3e-6, 0.05e-6, 1.0e5, 2.0e5, 0.0))
        for _ in range(8):
            o.step(1)
        runs[K] = o.particles()
    for K in (1, 10):
        for k in ("r", "z", "vr", "vt", "vz"):
            assert np.array_equal(runs[K][k], runs[None][k]), (K, k)


def test_heavy_subcycle_bookkeeping_and_stillness():
    """A full run with collisions and K = 10: charge and particle counts stay
    exact, and across a step that is not a heavy step no heavy particle
    moves (collisions change only velocities and labels)."""
    cfg = W.config("tiny", n_init=20_000)
    o = make_oracle(cfg)
    o.set_heavy_subcycle(10)
    o.inject(W.initial_population(cfg))
    off, inj = W.injection_schedule(cfg, 40)
    o.schedule_injection(off, inj)
    o.step(11)  # counters 0..10: the next step (counter 11) is not a heavy step
    before = o.particles()
    o.step(1)
    after = o.particles()
    hb = before["sp"] != W.E
    ha = after["sp"] != W.E
    ids, ib, ia = np.intersect1d(before["id"][hb], after["id"][ha], return_indices=True)
    assert len(ids) > 10_000
    assert np.array_equal(before["r"][hb][ib], after["r"][ha][ia])
    assert np.array_equal(before["z"][hb][ib], after["z"][ha][ia])
    o.step(28)
    d = o.diag()
    assert d["charge_alive"] + d["charge_absorbed"] == d["charge_injected"]
    assert int(np.sum(d["count"])) == d["n_alive"] == o.count()
    assert int(np.sum(d["events"])) > 0
