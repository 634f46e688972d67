"""Pins of the oracle's DSMC collisions: the event probability of Eq. 4, the
momentum/energy-conserving update of Eqs. 5-7 and the four stages of the
double-ionization scheme (Eqs. 11-15), plus the literal Eqs. 16-20."""
import numpy as np
import pytest
from scipy import stats

from conftest import make_oracle
from paper_2109_00214_amd import workload as W


def _uniform_vapour(cfg, n_cu_per_cell, n_cu1_per_cell, n_e_per_cell, v_e, seed,
                    n_cu2_per_tag=0, n_cu3_per_cell=0):
    """Cu (and Cu+, each Cu2+ tag, Cu3+) at rest, spread over every cell;
    monoenergetic electrons moving along +z, all with the same speed v_e."""
    rng = np.random.default_rng(seed)
    C = cfg.nr * cfg.nz
    dr, dz = cfg.R / cfg.nr, cfg.L / cfg.nz
    cells = np.arange(C)
    out = {k: [] for k in ("r", "z", "vr", "vt", "vz", "sp")}
    for cnt, sp, v in ((n_cu_per_cell, W.CU, 0.0), (n_cu1_per_cell, W.CU1, 0.0),
                       (n_cu2_per_tag, W.CU2_STEP, 0.0), (n_cu2_per_tag, W.CU2_DOUBLE, 0.0),
                       (n_cu2_per_tag, W.CU2_INIT, 0.0), (n_cu3_per_cell, W.CU3, 0.0),
                       (n_e_per_cell, W.E, v_e)):
        c = np.repeat(cells, cnt)
        i, j = c % cfg.nr, c // cfg.nr
        out["r"].append((i + 0.05 + 0.9 * rng.random(c.size)) * dr)
        out["z"].append((j + 0.05 + 0.9 * rng.random(c.size)) * dz)
        out["vr"].append(np.zeros(c.size))
        out["vt"].append(np.zeros(c.size))
        out["vz"].append(np.full(c.size, v))
        out["sp"].append(np.full(c.size, sp, np.uint8))
    return {k: np.concatenate(v) for k, v in out.items()}


@pytest.mark.parametrize("chain", [False, True])
def test_event_rate_matches_n_sigma_v(chain):
    """Monoenergetic beam in uniform Cu vapour (with chain=True also Cu2+ of
    every tag and Cu3+, and the channels on to Cu4+): the number of trials
    that pass the test of Eq. 4 equals sum(1 - exp(-dt v n_t sigma)) within
    3 sigma (binomial); channel shares follow x_k / X.  The Cu2+ density is
    that of all three tags together."""
    cfg = W.config("tiny", nr=8, nz=16, weight=1e3)
    sig = (3e-20, 2e-20, 0.5e-20, 4e-20) + ((2.5e-20, 1.5e-20) if chain else ())
    nch = len(sig)
    tables = W.constant_tables(sig)
    v_e = 2.0e6
    n_cu, n_cu1, n_e = 40, 20, 2
    n_cu2_tag, n_cu3 = (5, 10) if chain else (0, 0)
    n_target = {W.EL: n_cu, W.SI: n_cu, W.DI: n_cu, W.SI2: n_cu1, W.SI3: 3 * n_cu2_tag,
                W.SI4: n_cu3}
    expect_total = 0.0
    expect_ch = np.zeros(nch)
    got_total = 0
    got_ch = np.zeros(nch)
    for trial in range(12):
        c2 = W.config("tiny", nr=8, nz=16, weight=1e3, seed=100 + trial)
        o = make_oracle(c2, tables=tables)
        o.inject(_uniform_vapour(c2, n_cu, n_cu1, n_e, v_e, trial, n_cu2_tag, n_cu3))
        o.stage("sort")
        n = o.count()
        o.stage("collide")
        ch, tg, wn = o.collisions(n)
        d = o.diag()
        assert int(np.sum(d["events"])) + d["conflicts"] == int((ch > 0).sum())
        got_total += int((ch > 0).sum())
        got_ch += np.bincount(ch, minlength=W.NCHANNELS + 1)[1:nch + 1]
        assert np.bincount(ch, minlength=W.NCHANNELS + 1)[nch + 1:].sum() == 0
        _, vc = o.node_volumes()
        i = np.arange(c2.nr * c2.nz) % c2.nr
        xk = np.stack([c2.dt * v_e * (n_target[k] * c2.weight / vc[i]) * sig[k]
                       for k in range(nch)])
        X = xk.sum(axis=0)
        p = -np.expm1(-X)
        expect_total += n_e * p.sum()
        expect_ch += n_e * (xk / X * p).sum(axis=1)
    sd = np.sqrt(expect_total)
    assert abs(got_total - expect_total) < 3 * sd, (got_total, expect_total)
    for k in range(nch):
        assert abs(got_ch[k] - expect_ch[k]) < 3 * np.sqrt(expect_ch[k]) + 1, (k, got_ch, expect_ch)


def _collide_once(cfg, parts, tables=None):
    o = make_oracle(cfg, tables=tables)
    o.inject(parts)
    o.stage("sort")
    before = o.particles()
    n = o.count()
    o.stage("collide")
    after = o.particles()
    ch, tg, wn = o.collisions(n)
    return o, before, after, ch, tg, wn


def _ke(m, p, idx):
    return 0.5 * m * (p["vr"][idx] ** 2 + p["vt"][idx] ** 2 + p["vz"][idx] ** 2)


def _mom(m, p, idx):
    return m * np.array([p["vr"][idx], p["vt"][idx], p["vz"][idx]])


@pytest.mark.parametrize("channel", [W.EL, W.SI, W.DI, W.SI2, W.SI3, W.SI4])
def test_event_conservation_identities(channel):
    """Per event: EL conserves the pair's momentum and energy; ionizing
    events change the energy by -E_th + (m_e/2)|v_ion|^2 per stage-2
    electron and the momentum by m_e v_ion (the new electron inherits the
    ion's velocity, Eq. 13); the double-ionization split is orthogonal
    (Eq. 15: the velocities are the edges of a rectangle)."""
    cfg = W.config("tiny", nr=4, nz=8, weight=1e5)
    sig = [0.0] * W.NCHANNELS
    sig[channel] = 5e-19
    thr = list(W.THRESHOLDS_EV)
    tables = W.constant_tables(sig, thresholds=thr, n=4096)
    parts = _uniform_vapour(cfg, 30, 30, 2, 6.0e6, 1, n_cu2_per_tag=10, n_cu3_per_cell=30)
    rng = np.random.default_rng(2)
    for k in ("vr", "vt"):
        parts[k] = parts[k] + rng.normal(0, 1e5, parts[k].size) * (parts["sp"] == W.E)
        parts[k] = parts[k] + rng.normal(0, 600, parts[k].size) * (parts["sp"] != W.E)
    o, b, a, ch, tg, wn = _collide_once(cfg, parts, tables)
    Z, m = W.species_table()
    n = len(b["r"])
    winners = np.nonzero(wn)[0]
    assert len(winners) > 10
    created = n
    nev = 0
    for p in winners:
        assert ch[p] - 1 == channel
        t = tg[p]
        ke0 = _ke(W.ME, b, p) + _ke(W.M_CU, b, t)
        mo0 = _mom(W.ME, b, p) + _mom(W.M_CU, b, t)
        ke1 = _ke(W.ME, a, p) + _ke(W.M_CU, a, t)
        mo1 = _mom(W.ME, a, p) + _mom(W.M_CU, a, t)
        if channel == W.EL:
            assert a["sp"][t] == b["sp"][t]
            assert abs(ke1 - ke0) <= 1e-12 * ke0
            assert np.all(np.abs(mo1 - mo0) <= 1e-12 * np.abs(W.ME * 6e6))
            continue
        newb = [created] if channel != W.DI else [created, created + 1]
        created += len(newb)
        for q in newb:
            assert a["sp"][q] == W.E and a["id"][q] == b["id"].max() + 1 + (q - n)
            ke1 += _ke(W.ME, a, q)
            mo1 = mo1 + _mom(W.ME, a, q)
        vion = np.array([a["vr"][t], a["vt"][t], a["vz"][t]])
        thr_J = W.THRESHOLDS_EV[channel] * W.QE
        expect = ke0 - thr_J + 0.5 * W.ME * (vion @ vion)
        assert abs(ke1 - expect) <= 1e-12 * ke0
        assert np.all(np.abs(mo1 - (mo0 + W.ME * vion)) <= 1e-12 * W.ME * 6e6)
        assert b["sp"][t] in {W.SI: (W.CU,), W.DI: (W.CU,), W.SI2: (W.CU1,),
                              W.SI3: (W.CU2_STEP, W.CU2_DOUBLE, W.CU2_INIT),
                              W.SI4: (W.CU3,)}[channel]
        assert a["sp"][t] == {W.SI: W.CU1, W.DI: W.CU2_DOUBLE, W.SI2: W.CU2_STEP,
                              W.SI3: W.CU3, W.SI4: W.CU4}[channel]
        assert a["r"][newb[0]] == b["r"][t] and a["z"][newb[0]] == b["z"][t]
        if channel == W.DI:
            q6 = newb[1]
            assert a["r"][q6] == b["r"][p] and a["z"][q6] == b["z"][p]
            v5 = np.array([a["vr"][p], a["vt"][p], a["vz"][p]])
            v6 = np.array([a["vr"][q6], a["vt"][q6], a["vz"][q6]])
            assert abs(v5 @ v6) <= 1e-12 * (v5 @ v5 + v6 @ v6)
        nev += 1
    assert o.count() == created
    d = o.diag()
    assert d["events"][channel] == len(winners)


def test_claim_lowest_position_wins():
    cfg = W.config("tiny", nr=2, nz=2, weight=1e6)
    tables = W.constant_tables((1e-16, 0, 0, 0), n=4096)
    parts = _uniform_vapour(cfg, 2, 0, 20, 3.0e6, 4)
    o, b, a, ch, tg, wn = _collide_once(cfg, parts, tables)
    chosen = np.nonzero(ch)[0]
    assert len(chosen) > 20
    for t in np.unique(tg[chosen]):
        who = chosen[tg[chosen] == t]
        assert wn[who[0]] == 1 and np.all(wn[who[1:]] == 0)
    d = o.diag()
    # every passed trial is either a realized event or a lost claim
    assert d["conflicts"] == int((ch > 0).sum() - wn.sum())
    assert int(np.sum(d["events"])) == int(wn.sum())
    assert int(np.sum(d["events"])) + d["conflicts"] == int((ch > 0).sum())


def test_targets_are_uniform_in_cell():
    """Pairing picks every Cu in the electron's cell with equal probability."""
    tables = W.constant_tables((1e-15, 0, 0, 0), n=4096)
    counts = np.zeros(10)
    for trial in range(20):
        c2 = W.config("tiny", nr=2, nz=2, weight=1e8, seed=trial)
        parts = _uniform_vapour(c2, 10, 0, 200, 3.0e6, trial)
        o, b, a, ch, tg, wn = _collide_once(c2, parts, tables)
        off = o.offsets()
        C = 4
        e_cell = b["key"][: off[C]]
        for cell in range(C):
            sel = (ch[: off[C]] > 0) & (e_cell == cell)
            counts += np.bincount(tg[: off[C]][sel] - off[C + cell], minlength=10)
    assert stats.chisquare(counts).pvalue > 1e-3


def test_isotropic_directions():
    """Marsaglia's method gives unit vectors uniform on the sphere:
    cos(chi) uniform on [-1, 1], azimuth uniform on [0, 2 pi)."""
    cfg = W.config("tiny")
    o = make_oracle(cfg)
    n = np.array([o.isotropic(i, 2) for i in range(20000)])
    assert np.allclose(np.linalg.norm(n, axis=1), 1.0, atol=1e-15)
    assert stats.kstest(n[:, 2], stats.uniform(-1, 2).cdf).pvalue > 1e-3
    az = np.arctan2(n[:, 1], n[:, 0]) % (2 * np.pi)
    assert stats.kstest(az, stats.uniform(0, 2 * np.pi).cdf).pvalue > 1e-3
    # each purpose draws an independent stream
    m = np.array([o.isotropic(i, 3) for i in range(2000)])
    assert np.abs(np.mean(np.sum(n[:2000] * m, axis=1))) < 0.1


def test_rotation_matrix_eq20():
    rng = np.random.default_rng(3)
    from oracle import Oracle
    for _ in range(200):
        v = rng.normal(size=3)
        th = np.arccos(v[2] / np.linalg.norm(v))
        ph = np.arctan2(v[1], v[0])
        Rm = Oracle.rotation(th, ph)
        assert np.allclose(Rm @ Rm.T, np.eye(3), atol=1e-14)
        assert np.allclose(Rm @ v, [0, 0, np.linalg.norm(v)], atol=1e-14 * np.linalg.norm(v))


def test_split_literal_vs_projection_form():
    """The literal Eqs. 16-19 with cos(chi) ~ U[0,1), psi ~ U[0, 2 pi) and
    the projection form v5 = (v.n) n with n uniform on the sphere give the
    same distribution of (v5, v6)."""
    from oracle import Oracle
    rng = np.random.default_rng(9)
    cfg = W.config("tiny")
    o = make_oracle(cfg)
    lit, proj = [], []
    v = np.array([1.0e6, -2.0e6, 0.5e6])
    vm = np.linalg.norm(v)
    for i in range(4000):
        chi = np.arccos(rng.random())
        psi = 2 * np.pi * rng.random()
        v5 = Oracle.split_literal(v, chi, psi)
        v6 = v - v5
        assert abs(v5 @ v6) <= 1e-9 * vm * vm
        assert abs(np.linalg.norm(v5) - np.cos(chi) * vm) <= 1e-9 * vm
        lit.append(v5)
        nh = o.isotropic(i, 4)
        proj.append((v @ nh) * nh)
    lit, proj = np.array(lit), np.array(proj)
    for f in (lambda x: np.linalg.norm(x, axis=1) / vm, lambda x: x[:, 0], lambda x: x[:, 2]):
        assert stats.ks_2samp(f(lit), f(proj)).pvalue > 1e-3
    # along the z axis (theta = 0) the frame is still well defined
    v5 = Oracle.split_literal(np.array([0.0, 0.0, 3.0]), 0.3, 1.0)
    assert abs(np.linalg.norm(v5) - 3.0 * np.cos(0.3)) < 1e-12


def test_cross_section_table_lookup():
    """Linear interpolation in sqrt(E), zero below threshold, clamp at end."""
    cfg = W.config("tiny")
    tabs = W.cross_section_tables()
    o = make_oracle(cfg, tables=tabs)
    mr = W.ME * W.M_CU / (W.ME + W.M_CU)
    for ch, thr, dsq, sig in tabs:
        for E in (0.5, 7.0, 7.8, 20.0, 27.9, 28.5, 150.0, 1000.0, 9000.0):
            g = np.sqrt(2 * E * W.QE / mr)
            s = o.cross_section(ch, g)
            if E < thr * (1 - 1e-12):
                assert s == 0.0
                continue
            x = np.sqrt(E) / dsq
            if x >= len(sig) - 1:
                assert s == sig[-1]
            else:
                i = int(x)
                ref = sig[i] + (x - i) * (sig[i + 1] - sig[i])
                assert abs(s - ref) <= 1e-9 * max(abs(ref), 1e-30)
                ref_lotz = {W.EL: 1e-19 / (1 + E / 20)}.get(ch)
                if ref_lotz is not None:
                    assert abs(s - ref_lotz) < 1e-3 * ref_lotz


def test_cu2_targets_are_uniform_over_the_tags():
    """The Cu2+ target of the Cu2+ -> Cu3+ channel is drawn uniformly from
    the Cu2+ of every tag in the cell: each of the 15 Cu2+ of a cell (5 per
    tag) is picked equally often, and each tag's share of the events is a
    third."""
    sig = [0.0] * W.NCHANNELS
    sig[W.SI3] = 1e-15
    tables = W.constant_tables(sig, n=4096)
    counts = np.zeros(15)
    tags = np.zeros(3)
    for trial in range(20):
        c2 = W.config("tiny", nr=2, nz=2, weight=1e8, seed=trial)
        parts = _uniform_vapour(c2, 0, 0, 200, 3.0e6, trial, n_cu2_per_tag=5)
        o, b, a, ch, tg, wn = _collide_once(c2, parts, tables)
        off = o.offsets()
        C = 4
        e_cell = b["key"][: off[C]]
        for cell in range(C):
            sel = (ch[: off[C]] > 0) & (e_cell == cell)
            assert np.all(ch[: off[C]][sel] == W.SI3 + 1)
            pick = tg[: off[C]][sel]
            assert np.all((pick >= off[3 * C + cell]) & (pick < off[3 * C + cell + 1]))
            counts += np.bincount(pick - off[3 * C + cell], minlength=15)
            tags += np.bincount(b["sp"][pick] - W.CU2_STEP, minlength=3)
    assert stats.chisquare(counts).pvalue > 1e-3
    assert stats.chisquare(tags).pvalue > 1e-3


def test_chain_channels_absent_without_tables():
    """Without tables for Cu2+ -> Cu3+ and Cu3+ -> Cu4+, a run with Cu2+ and
    Cu3+ present is bit-identical to one whose two tables hold zeros (the
    draws, sums and choices of the other channels are untouched), and no
    Cu3+ or Cu4+ is made."""
    cfg = W.config("tiny", n_init=20_000)
    parts = W.initial_population(cfg)
    tabs4 = W.cross_section_tables()
    zero = [(W.SI3, 36.84, 2.0 ** -4, np.zeros(1025)), (W.SI4, 57.38, 2.0 ** -4, np.zeros(1025))]
    runs = []
    for tabs in (tabs4, tabs4 + zero):
        o = make_oracle(cfg, tables=tabs)
        o.inject(parts)
        o.step(30)
        runs.append((o.particles(), o.diag()))
    for k in runs[0][0]:
        assert np.array_equal(runs[0][0][k], runs[1][0][k]), k
    for d, _ in ((runs[0][1], 0), (runs[1][1], 1)):
        assert d["count"][W.CU3] == 0 and d["count"][W.CU4] == 0
        assert d["events"][W.SI3] == 0 and d["events"][W.SI4] == 0
    assert int(np.sum(runs[0][1]["events"])) > 0


def test_chain_run_bookkeeping():
    """A run with the whole chain on: Cu3+ and Cu4+ appear, every event of
    Cu2+ -> Cu3+ and Cu3+ -> Cu4+ makes one electron, and the charge and
    particle counts stay exact."""
    cfg = W.config("tiny", nr=8, nz=16, weight=1e5)
    tables = W.constant_tables([3e-19] * W.NCHANNELS, thresholds=list(W.THRESHOLDS_EV), n=4096)
    o = make_oracle(cfg, tables=tables)
    parts = _uniform_vapour(cfg, 20, 10, 4, 6.0e6, 3, n_cu2_per_tag=4, n_cu3_per_cell=8)
    rng = np.random.default_rng(8)
    e = parts["sp"] == W.E
    parts["vr"] = np.where(e, rng.normal(0.0, 1e6, e.size), parts["vr"])  # electron pairs move apart
    o.inject(parts)
    o.step(6)
    d = o.diag()
    assert np.all(d["events"] > 0), d["events"]
    assert d["count"][W.CU4] > 0
    assert d["created"] == (d["events"][W.SI] + 2 * d["events"][W.DI] + d["events"][W.SI2] +
                            d["events"][W.SI3] + d["events"][W.SI4])
    assert d["charge_alive"] + d["charge_absorbed"] == d["charge_injected"]
    assert int(np.sum(d["count"])) == d["n_alive"] == o.count()


def test_literal_split_run_mode():
    """With the literal Eqs. 16-20 as the double ionization's last stage, the
    two electrons it leaves are the edges of a rectangle whose diagonal is
    the electron before it (v5 + v6 = v3, v5 . v6 = 0) and |v5| / |v3| =
    cos(chi) is uniform on [0, 1)."""
    cfg = W.config("tiny", nr=4, nz=8, weight=1e5)
    sig = [0.0] * W.NCHANNELS
    sig[W.DI] = 5e-19
    tables = W.constant_tables(sig, thresholds=list(W.THRESHOLDS_EV), n=4096)
    ratios = []
    for trial in range(6):
        c2 = W.config("tiny", nr=4, nz=8, weight=1e5, seed=300 + trial)
        o = make_oracle(c2, tables=tables)
        o.set_split_literal(True)
        parts = _uniform_vapour(c2, 30, 0, 3, 6.0e6, trial)
        o.inject(parts)
        o.stage("sort")
        n = o.count()
        o.stage("collide")
        a = o.particles()
        ch, tg, wn = o.collisions(n)
        win = np.nonzero(wn)[0]
        # the stage-4 electron of winner k is the (2k+1)-th created particle
        for k, p in enumerate(win):
            q6 = n + 2 * k + 1
            v5 = np.array([a["vr"][p], a["vt"][p], a["vz"][p]])
            v6 = np.array([a["vr"][q6], a["vt"][q6], a["vz"][q6]])
            v3 = v5 + v6
            m = np.linalg.norm(v3)
            assert abs(v5 @ v6) <= 1e-9 * m * m
            ratios.append(np.linalg.norm(v5) / m)
    assert len(ratios) > 200
    assert stats.kstest(ratios, "uniform").pvalue > 1e-3
