"""Seeded synthetic inputs shaped like the paper's cathode-spot workload.

This module holds none of the method's arithmetic: it only draws particles
and builds the cross-section tables that both the GPU library and the CPU
oracle receive as inputs (positions, velocities at the half step before
their first push, species, and sigma tables uniform in sqrt(E)).

Workload recipe (paper Sec. 2.3, rescaled to the benchmark domains):
  * domain: r in [0, R), z in [0, L), gap L = 2 um, R = L * nr / nz;
    cathode at z = 0 held at -V, grounded anode at z = L, V = 2.9 kV
    (the source voltage of the paper's circuit);
  * initial population: 40 % e, 40 % Cu, 18 % Cu+, 2 % Cu2+ (tag INIT);
    density falls off as exp(-d / 0.25 um) with d the distance to the
    cathode spot disk (r <= 0.5 um, z = 0); electrons 95 % Maxwellian at
    5 eV plus a 5 % 100 eV beam along +z; heavy particles Maxwellian 2000 K;
  * injection every step at the spot: electrons (field emission at a
    constant rate) and neutral Cu at 3 % of the electron rate (the paper's
    neutral-to-electron flux ratio), both flux-Maxwellian at 2000 K,
    spread over the first step of flight;
  * cross sections: synthetic Lotz-form ionization tables with the
    thresholds 7.73 eV (Cu -> Cu+), 20.29 eV (Cu+ -> Cu2+), 28.0 eV
    (Cu -> Cu2+, direct double ionization) and a synthetic elastic
    table; the paper's own data (its Fig. 1) are not available.
"""
from dataclasses import dataclass, replace

import numpy as np

# CODATA 2018
QE = 1.602176634e-19
ME = 9.1093837015e-31
AMU = 1.66053906660e-27
KB = 1.380649e-23
EPS0 = 8.8541878128e-12
M_CU = 63.546 * AMU

# species enum: E, CU, CU1, CU2_STEP, CU2_DOUBLE, CU2_INIT, CU3, CU4
E, CU, CU1, CU2_STEP, CU2_DOUBLE, CU2_INIT, CU3, CU4 = range(8)
NSPECIES = 8
SPECIES_NAMES = ("e", "Cu", "Cu+", "Cu2+(step)", "Cu2+(double)", "Cu2+(init)", "Cu3+", "Cu4+")
# channels: electron impact (six), the heavy projectiles' charge exchange
# (Cu+ + Cu) and neutral-neutral elastic (Cu + Cu), the Coulomb collisions of
# electrons with Cu+ and with electrons; every channel from SI3 on takes part
# only when its table is given
EL, SI, DI, SI2, SI3, SI4, CEX, NN, CEI, CEE = range(10)
NCHANNELS = 10
CHANNEL_NAMES = ("elastic", "Cu->Cu+", "Cu->Cu2+ (double)", "Cu+->Cu2+", "Cu2+->Cu3+",
                 "Cu3+->Cu4+", "Cu+ + Cu charge exchange", "Cu + Cu elastic", "e + Cu+ Coulomb",
                 "e + e Coulomb")
# ionization energies (eV) of Cu, Cu+, Cu2+, Cu3+ and the paper's double-
# ionization threshold; the other channels lose no energy
THRESHOLDS_EV = (0.0, 7.73, 28.0, 20.29, 36.84, 57.38, 0.0, 0.0, 0.0, 0.0)


def species_table():
    """Charge numbers and masses, enum order (every Cu state has M_Cu)."""
    Z = np.array([-1, 0, 1, 2, 2, 2, 3, 4], dtype=np.int32)
    m = np.array([ME] + [M_CU] * 7, dtype=np.float64)
    return Z, m


def lotz(E, P, q, a_cm2=4.5e-14):
    """Simplified Lotz form sigma = a q ln(E/P) / (E P) in m^2 (E, P in eV)."""
    E = np.asarray(E, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        s = a_cm2 * q * np.log(np.where(E > P, E / P, 1.0)) / (np.where(E > 0, E, 1.0) * P)
    return np.where(E >= P, s, 0.0) * 1e-4


def coulomb_sigma(E, ln_lambda=10.0, E_min=0.1):
    """Momentum-transfer cross section of a Coulomb pair of unit charges,
    4 pi lnL b^2 with b = e^2 / (8 pi eps0 E) (E the energy of relative motion
    in eV, held at E_min below it), in m^2."""
    E = np.maximum(np.asarray(E, dtype=np.float64), E_min)
    b = QE / (8.0 * np.pi * EPS0 * E)
    return 4.0 * np.pi * ln_lambda * b * b


def cross_section_tables(dsqrtE=2.0 ** -4, n=1025, chain=False, heavy=False, coulomb=False):
    """(channel, threshold_eV, dsqrtE, sigma[n]) for EL, SI, DI, SI2, with
    chain=True also SI3 and SI4 (Lotz forms with 9 and 8 d electrons), with
    heavy=True also CEX and NN (stand-ins: a resonant charge-exchange form
    (a - b ln E)^2, a = 7.5 A, b = 0.4 A, E >= 0.01 eV; hard spheres of
    diameter 2.6 A).

    With coulomb=True also CEI and CEE (coulomb_sigma, ln Lambda = 10).
    Tables are uniform in sqrt(E/eV) with spacing dsqrtE (a power of 2); E is
    the energy of relative motion of the pair.
    """
    sq = np.arange(n, dtype=np.float64) * dsqrtE
    En = sq * sq
    el = 1e-19 / (1.0 + En / 20.0)
    si = lotz(En, 7.73, 1.0)
    di = lotz(En, 28.0, 1.0)
    si2 = lotz(En, 20.29, 10.0)
    out = [(EL, 0.0, dsqrtE, el), (SI, 7.73, dsqrtE, si), (DI, 28.0, dsqrtE, di),
           (SI2, 20.29, dsqrtE, si2)]
    if chain:
        out += [(SI3, 36.84, dsqrtE, lotz(En, 36.84, 9.0)), (SI4, 57.38, dsqrtE, lotz(En, 57.38, 8.0))]
    if heavy:
        cex = (7.5 - 0.4 * np.log(np.maximum(En, 0.01))) ** 2 * 1e-20
        nn = np.full(n, np.pi * 2.6e-10 ** 2)
        out += [(CEX, 0.0, dsqrtE, cex), (NN, 0.0, dsqrtE, nn)]
    if coulomb:
        out += [(CEI, 0.0, dsqrtE, coulomb_sigma(En)), (CEE, 0.0, dsqrtE, coulomb_sigma(En))]
    return out


def constant_tables(sig, dsqrtE=2.0 ** -4, n=64, thresholds=None):
    """Constant-sigma tables (rate tests); sig = one value per channel given
    (4: the paper's four channels, 6: with the chain to Cu4+)."""
    thresholds = thresholds or (0.0,) * len(sig)
    return [(k, float(thresholds[k]), dsqrtE, np.full(n, float(sig[k]))) for k in range(len(sig))]


@dataclass(frozen=True)
class Config:
    name: str
    nr: int
    nz: int
    L: float = 2e-6
    V: float = 2900.0
    dt: float = 1e-14
    weight: float = 100.0
    seed: int = 1
    n_init: int = 50_000
    inj_e: int = 100
    inj_cu: int = 3
    steps: int = 200
    spot: float = 0.5e-6
    lam: float = 0.25e-6
    enable_di: bool = True

    @property
    def R(self):
        return self.L * self.nr / self.nz


CONFIGS = {
    # plain FP64, 32x64 cells, 50k particles, W = 100, 200 steps, seed 1
    "tiny": Config("tiny", 32, 64),
    # paper-shaped: 256x512 cells, 5M particles, W = 1, 2000 steps
    "paper": Config("paper", 256, 512, weight=1.0, n_init=5_000_000, inj_e=10_000,
                    inj_cu=300, steps=2000),
}


def config(name, **kw):
    return replace(CONFIGS[name], **kw)


def run_capacity(cfg, nsteps):
    """Particle capacity of a run of nsteps: the initial population with a
    quarter to spare, every scheduled neutral, forty steps' worth of emitted
    electrons (they leave the gap within a few tens of steps) and a fixed
    margin for the electrons the collisions create."""
    return int(1.25 * cfg.n_init + cfg.inj_cu * nsteps + 40 * cfg.inj_e + 1_000_000)


def _rng(seed, tag):
    return np.random.Generator(np.random.Philox(key=[int(seed), int(tag)]))


def _positions(rng, n, cfg):
    """n positions with density ~ exp(-d/lam), d = distance to the spot disk."""
    R, L, lam, rs = cfg.R, cfg.L, cfg.lam, cfg.spot
    out_r = np.empty(0)
    out_z = np.empty(0)
    while out_r.size < n:
        m = max(1024, int((n - out_r.size) * 2.6))
        # z from an exponential truncated to [0, L); r uniform in area
        u = rng.random(m)
        z = -lam * np.log1p(-u * (1.0 - np.exp(-L / lam)))
        r = R * np.sqrt(rng.random(m))
        d = np.where(r <= rs, z, np.sqrt((r - rs) ** 2 + z ** 2))
        acc = rng.random(m) < np.exp(-(d - z) / lam)
        ok = acc & (r < R) & (z < L) & (z >= 0)
        out_r = np.concatenate([out_r, r[ok]])
        out_z = np.concatenate([out_z, z[ok]])
    return out_r[:n], out_z[:n]


def initial_population(cfg, n=None, mix=(0.40, 0.40, 0.18, 0.02)):
    """Initial super-particles (v at the half step before the first push)."""
    n = cfg.n_init if n is None else n
    rng = _rng(cfg.seed, 0x1A17)  # stream INIT
    counts = [int(round(n * f)) for f in mix]
    counts[0] += n - sum(counts)
    sp = np.concatenate([np.full(c, s, np.uint8)
                         for c, s in zip(counts, (E, CU, CU1, CU2_INIT))])
    r, z = _positions(rng, n, cfg)
    v = np.zeros((3, n))
    ne = counts[0]
    s_e = np.sqrt(5.0 * QE / ME)
    s_h = np.sqrt(KB * 2000.0 / M_CU)
    v[:, :ne] = rng.normal(0.0, s_e, (3, ne))
    beam = rng.random(ne) < 0.05
    v[:, :ne][:, beam] = 0.0
    v[2, :ne][beam] = np.sqrt(2.0 * 100.0 * QE / ME)
    v[:, ne:] = rng.normal(0.0, s_h, (3, n - ne))
    return {"r": r, "z": z, "vr": v[0].copy(), "vt": v[1].copy(), "vz": v[2].copy(),
            "sp": sp}


def _emit(rng, n, mass, cfg):
    s = np.sqrt(KB * 2000.0 / mass)
    r = cfg.spot * np.sqrt(rng.random(n))
    vz = s * np.sqrt(-2.0 * np.log1p(-rng.random(n)))  # flux-weighted normal component
    vr = rng.normal(0.0, s, n)
    vt = rng.normal(0.0, s, n)
    z = rng.random(n) * vz * cfg.dt
    return r, z, vr, vt, vz


def injection_schedule(cfg, nsteps, first_step=0):
    """Per-step injection lists for steps first_step .. first_step+nsteps-1.

    Returns (offsets[nsteps+1], particle dict) in injection order: per step
    the electrons, then the neutrals.
    """
    parts = {k: [] for k in ("r", "z", "vr", "vt", "vz", "sp")}
    offs = [0]
    for s in range(first_step, first_step + nsteps):
        rng = _rng(cfg.seed, 0x10000000 + s)  # stream INJ, one per step
        for cnt, spc, mass in ((cfg.inj_e, E, ME), (cfg.inj_cu, CU, M_CU)):
            r, z, vr, vt, vz = _emit(rng, cnt, mass, cfg)
            for k, a in zip(("r", "z", "vr", "vt", "vz"), (r, z, vr, vt, vz)):
                parts[k].append(a)
            parts["sp"].append(np.full(cnt, spc, np.uint8))
        offs.append(offs[-1] + cfg.inj_e + cfg.inj_cu)
    out = {k: (np.concatenate(v) if v else np.zeros(0)) for k, v in parts.items()}
    out["sp"] = out["sp"].astype(np.uint8)
    return np.array(offs, dtype=np.int64), out


def subset(parts, idx):
    return {k: np.ascontiguousarray(v[idx]) for k, v in parts.items()}


# ---------------------------------------------------------------------------
# learned Poisson part: initial weights of the U-Net (seeded He-normal), in the
# layer order of the library's flat weight vector
def unet_layer_shapes(levels=4, base=16, cin=2):
    """(c_out, c_in, k) per layer: encoder levels, decoder levels from the
    bottom up to level 0, then the 1x1 output layer."""
    out, prev = [], cin
    for l in range(levels):
        c = base << l
        out += [(c, prev, 3), (c, c, 3)]
        prev = c
    for l in range(levels - 2, -1, -1):
        c = base << l
        out += [(c, c + (base << (l + 1)), 3), (c, c, 3)]
    out.append((1, base, 1))
    return out


def unet_init_weights(levels=4, base=16, seed=1):
    rng = np.random.Generator(np.random.Philox(key=[seed, 0x4E4554]))
    parts = []
    for co, ci, k in unet_layer_shapes(levels, base):
        std = np.sqrt(2.0 / (ci * k * k)) if k == 3 else np.sqrt(1.0 / ci)
        parts.append(rng.normal(0.0, std, size=co * k * k * ci))
    return np.concatenate(parts).astype(np.float32)


# ---------------------------------------------------------------------------
# batched ensemble: uneven replicas (grid 128x256 or 256x512 with p = 1/2,
# cathode voltage uniform in 1-5 kV, particle count log-uniform in
# [0.2M, 8M], seed 1000 + k, weight 5e6 / N so every replica carries the same
# real charge, injection scaled with N from the paper-shaped rates)
def ensemble_configs(n=48, seed=1000, nmin=200_000, nmax=8_000_000):
    rng = _rng(seed, 0xE45E)
    out = []
    for k in range(n):
        big = rng.random() < 0.5
        V = 1000.0 + 4000.0 * rng.random()
        N = int(round(np.exp(np.log(nmin) + (np.log(nmax) - np.log(nmin)) * rng.random())))
        f = N / 5_000_000
        out.append(Config("ensemble-%d" % k, 256 if big else 128, 512 if big else 256, V=V,
                          weight=5e6 / N, seed=seed + k, n_init=N,
                          inj_e=max(1, int(round(10_000 * f))), inj_cu=max(1, int(round(300 * f)))))
    return out
