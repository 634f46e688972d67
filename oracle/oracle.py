"""ctypes wrapper of the oracle library (test infrastructure only).

Argument marshalling only; every step of the method is computed in
``pd_oracle.c``.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pd_oracle.c")
_LIB = os.path.join(_HERE, "libpd_oracle.so")

NSPECIES = 8
NKEYS = 6
NCHANNELS = 10


def build_oracle(force=True):
    """Compile the oracle with gcc, FP64, no contraction, no fast-math."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("n_alive", C.c_int64), ("next_id", C.c_int64),
                ("count", C.c_int64 * NSPECIES), ("events", C.c_int64 * NCHANNELS),
                ("conflicts", C.c_int64), ("created", C.c_int64),
                ("absorbed", (C.c_int64 * NSPECIES) * 3), ("injected", C.c_int64 * NSPECIES),
                ("charge_alive", C.c_int64), ("charge_absorbed", C.c_int64),
                ("charge_injected", C.c_int64), ("ke_J", C.c_double * NSPECIES),
                ("gamma", C.c_double), ("qbar", C.c_double),
                ("spectrum", (C.c_int64 * 66) * 3), ("V_gap", C.c_double),
                ("emitted", C.c_int64 * 2), ("sputtered", C.c_int64),
                ("real", C.c_int64 * NSPECIES)]


_lib = None


def oracle_lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_oracle(force=False)
        _lib = load_oracle(_LIB)
    return _lib


def load_oracle(path):
    """A ctypes handle of an oracle library built at ``path`` (the tests that
    check that a pin catches a planted mistake load mutated copies this way)."""
    lib = C.CDLL(path)
    P = C.c_void_p
    dp = C.POINTER(C.c_double)
    lib.or_create.restype = P
    lib.or_create.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                              C.c_double, C.c_double, C.c_uint64, C.c_int, C.c_int, C.c_int]
    lib.or_destroy.argtypes = [P]
    lib.or_last_error.restype = C.c_char_p
    lib.or_set_species.argtypes = [P, C.c_int, P, P]
    lib.or_set_cross_section.argtypes = [P, C.c_int, C.c_double, C.c_int, C.c_double, P]
    lib.or_inject.argtypes = [P, C.c_int64, P, P, P, P, P, P]
    lib.or_inject_weighted.argtypes = [P, C.c_int64, P, P, P, P, P, P, P]
    lib.or_get_weights.argtypes = [P, P]
    lib.or_schedule_injection.argtypes = [P, C.c_int, P, P, P, P, P, P, P]
    lib.or_step.argtypes = [P, C.c_int]
    lib.or_set_heavy_subcycle.argtypes = [P, C.c_int]
    lib.or_set_emission.argtypes = [P] + [C.c_double] * 5
    lib.or_set_circuit.argtypes = [P] + [C.c_double] * 3
    lib.or_set_split_literal.argtypes = [P, C.c_int]
    lib.or_set_sputtering.argtypes = [P, C.c_int]
    lib.or_sputter_yield.restype = C.c_double
    lib.or_sputter_yield.argtypes = [C.c_double]
    for nm in ("sort", "collide", "deposit", "poisson", "field", "push",
               "compact_inject", "end"):
        getattr(lib, "or_stage_" + nm).argtypes = [P]
    lib.or_count.restype = C.c_int64
    lib.or_count.argtypes = [P]
    lib.or_get_particles.argtypes = [P] + [P] * 8
    lib.or_set_velocities.argtypes = [P, P, P, P]
    lib.or_get_field.argtypes = [P, P, P, P, P]
    lib.or_set_charge.argtypes = [P, P]
    lib.or_set_potential.argtypes = [P, P]
    lib.or_get_offsets.argtypes = [P, P]
    lib.or_get_collisions.argtypes = [P, P, P, P]
    lib.or_get_diag.argtypes = [P, C.POINTER(_Diag)]
    lib.or_philox4x32_10.argtypes = [P, P, P]
    lib.or_poisson_solve.argtypes = [P, P, P]
    lib.or_poisson_residual.argtypes = [P, P, P, dp, dp]
    lib.or_poisson_residual.restype = None
    lib.or_isotropic.argtypes = [P, C.c_uint32, C.c_uint32, P]
    lib.or_rotation.argtypes = [C.c_double, C.c_double, P]
    lib.or_split_literal.argtypes = [P, C.c_double, C.c_double, P]
    lib.or_node_volumes.argtypes = [P, P, P]
    lib.or_cross_section.restype = C.c_double
    lib.or_cross_section.argtypes = [P, C.c_int, C.c_double]
    del dp
    return lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def philox4x32_10(ctr, key):
    """Philox4x32-10 block: ctr = 4 uint32 words, key = 2 uint32 words."""
    lib = oracle_lib()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib.or_philox4x32_10(_p(c), _p(k), _p(o))
    return o


class Oracle:
    """One oracle simulation (mirrors the C-ABI calls of the GPU library)."""

    def __init__(self, nr, nz, R, L, V, dt, weight, seed, enable_di=True,
                 deposit_off=False, collisions_off=False, lib=None):
        self.lib = oracle_lib() if lib is None else lib
        self.nr, self.nz = nr, nz
        self.R, self.L, self.V, self.dt, self.weight, self.seed = R, L, V, dt, weight, seed
        h = self.lib.or_create(nr, nz, R, L, V, dt, weight, seed, int(enable_di),
                               int(deposit_off), int(collisions_off))
        if not h:
            raise ValueError(self.lib.or_last_error().decode())
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.or_destroy(h)
            self.h = None

    def _chk(self, rc):
        if rc != 0:
            raise ValueError(self.lib.or_last_error().decode())

    def set_species(self, Z, mass):
        Z = np.ascontiguousarray(Z, dtype=np.int32)
        m = np.ascontiguousarray(mass, dtype=np.float64)
        self._chk(self.lib.or_set_species(self.h, len(Z), _p(Z), _p(m)))

    def set_cross_section(self, channel, threshold_eV, dsqrtE, sigma):
        s = np.ascontiguousarray(sigma, dtype=np.float64)
        self._chk(self.lib.or_set_cross_section(self.h, channel, threshold_eV, len(s),
                                                dsqrtE, _p(s)))

    @staticmethod
    def _arrs(parts):
        return [np.ascontiguousarray(parts[k], dtype=np.float64)
                for k in ("r", "z", "vr", "vt", "vz")] + [
            np.ascontiguousarray(parts["sp"], dtype=np.uint8)]

    def inject(self, parts, mult=None):
        """append particles; mult (optional): each one's multiplicity, the
        number of W-weight units it stands for (unequal weights)"""
        a = self._arrs(parts)
        if mult is None:
            self._chk(self.lib.or_inject(self.h, len(a[0]), *[_p(x) for x in a]))
        else:
            m = np.ascontiguousarray(mult, dtype=np.uint16)
            assert len(m) == len(a[0])
            self._chk(self.lib.or_inject_weighted(self.h, len(a[0]), *[_p(x) for x in a],
                                                  _p(m)))

    def weights(self):
        """the multiplicities, in the order of particles()"""
        out = np.zeros(self.count(), np.uint16)
        self.lib.or_get_weights(self.h, _p(out))
        return out

    def schedule_injection(self, offsets, parts):
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        a = self._arrs(parts)
        self._chk(self.lib.or_schedule_injection(self.h, len(off) - 1, _p(off),
                                                 *[_p(x) for x in a]))

    def set_heavy_subcycle(self, every):
        self._chk(self.lib.or_set_heavy_subcycle(self.h, int(every)))

    def set_emission(self, beta, r_tip, phi_w, neutral_ratio, T):
        self._chk(self.lib.or_set_emission(self.h, beta, r_tip, phi_w, neutral_ratio, T))

    def set_circuit(self, V0, R, C):
        self._chk(self.lib.or_set_circuit(self.h, V0, R, C))

    def set_split_literal(self, on):
        self._chk(self.lib.or_set_split_literal(self.h, 1 if on else 0))

    def set_sputtering(self, on):
        self._chk(self.lib.or_set_sputtering(self.h, 1 if on else 0))

    @staticmethod
    def sputter_yield(E_eV):
        return oracle_lib().or_sputter_yield(E_eV)

    def step(self, nsteps=1):
        self._chk(self.lib.or_step(self.h, nsteps))

    def stage(self, name):
        getattr(self.lib, "or_stage_" + name)(self.h)

    def count(self):
        return int(self.lib.or_count(self.h))

    def particles(self):
        n = self.count()
        out = {k: np.zeros(n, np.float64) for k in ("r", "z", "vr", "vt", "vz")}
        out["sp"] = np.zeros(n, np.uint8)
        out["id"] = np.zeros(n, np.uint32)
        out["key"] = np.zeros(n, np.uint32)
        self.lib.or_get_particles(self.h, *[_p(out[k]) for k in
                                            ("r", "z", "vr", "vt", "vz", "sp", "id", "key")])
        return out

    def set_velocities(self, vr, vt, vz):
        a = [np.ascontiguousarray(x, dtype=np.float64) for x in (vr, vt, vz)]
        assert all(len(x) == self.count() for x in a)
        self.lib.or_set_velocities(self.h, *[_p(x) for x in a])

    def field(self):
        nn = (self.nr + 1) * (self.nz + 1)
        shp = (self.nz + 1, self.nr + 1)
        phi, Er, Ez = (np.zeros(nn) for _ in range(3))
        Q = np.zeros(nn, np.int64)
        self.lib.or_get_field(self.h, _p(phi), _p(Er), _p(Ez), _p(Q))
        return {"phi": phi.reshape(shp), "Er": Er.reshape(shp), "Ez": Ez.reshape(shp),
                "Q": Q.reshape(shp)}

    def set_charge(self, Q):
        q = np.ascontiguousarray(Q, dtype=np.int64).reshape(-1)
        assert q.size == (self.nr + 1) * (self.nz + 1)
        self.lib.or_set_charge(self.h, _p(q))

    def set_potential(self, phi):
        f = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1)
        assert f.size == (self.nr + 1) * (self.nz + 1)
        self.lib.or_set_potential(self.h, _p(f))

    def offsets(self):
        o = np.zeros(NKEYS * self.nr * self.nz + 1, np.int64)
        self.lib.or_get_offsets(self.h, _p(o))
        return o

    def collisions(self, n):
        ch = np.zeros(n, np.uint8)
        tg = np.zeros(n, np.uint32)
        wn = np.zeros(n, np.uint8)
        self.lib.or_get_collisions(self.h, _p(ch), _p(tg), _p(wn))
        return ch, tg, wn

    def diag(self):
        d = _Diag()
        self.lib.or_get_diag(self.h, C.byref(d))
        out = {}
        for name, _ in _Diag._fields_:
            v = getattr(d, name)
            if isinstance(v, (int, float)):
                out[name] = v
            else:
                out[name] = np.array([list(x) if not isinstance(x, (int, float)) else x
                                      for x in v])
        return out

    def poisson_solve(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        out = np.zeros_like(f)
        self.lib.or_poisson_solve(self.h, _p(f), _p(out))
        return out.reshape(self.nz + 1, self.nr + 1)

    def poisson_residual(self, Q, phi):
        """(||b - A phi||, ||b||) of the volume-weighted Poisson system."""
        q = np.ascontiguousarray(Q, dtype=np.int64).reshape(-1)
        f = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1)
        assert q.size == f.size == (self.nr + 1) * (self.nz + 1)
        rn, bn = C.c_double(), C.c_double()
        self.lib.or_poisson_residual(self.h, _p(q), _p(f), C.byref(rn), C.byref(bn))
        return rn.value, bn.value

    def isotropic(self, pid, purpose):
        n = np.zeros(3)
        self.lib.or_isotropic(self.h, pid, purpose, _p(n))
        return n

    def node_volumes(self):
        vn = np.zeros(self.nr + 1)
        vc = np.zeros(self.nr)
        self.lib.or_node_volumes(self.h, _p(vn), _p(vc))
        return vn, vc

    def cross_section(self, channel, g):
        return self.lib.or_cross_section(self.h, channel, g)

    @staticmethod
    def rotation(theta, phi):
        m = np.zeros(9)
        oracle_lib().or_rotation(theta, phi, _p(m))
        return m.reshape(3, 3)

    @staticmethod
    def split_literal(v, chi, psi):
        v = np.ascontiguousarray(v, dtype=np.float64)
        o = np.zeros(3)
        oracle_lib().or_split_literal(_p(v), chi, psi, _p(o))
        return o
