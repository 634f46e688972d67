"""Thin ctypes binding of the gfx950 PIC-DSMC library (include/pd.h).

Argument marshalling only: the functions below carry the C names and pass
host numpy arrays straight through; every step of the method runs in the
library's HIP kernels.  There is no CPU fallback: if ``libpd.so`` is missing
or no GPU is present, the calls raise.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpd.so")

PD_OK, PD_EINVAL, PD_ENOMEM, PD_EDEVICE, PD_ESTATE, PD_ENOCONV, PD_ECAPACITY = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "PD_OK", -1: "PD_EINVAL", -2: "PD_ENOMEM", -3: "PD_EDEVICE", -4: "PD_ESTATE",
                -5: "PD_ENOCONV", -6: "PD_ECAPACITY"}
PD_FP64_DET, PD_FP32_MIXED = 0, 1
PD_POISSON_DIRECT64, PD_POISSON_MGPCG, PD_POISSON_LEARNED, PD_POISSON_SPECTRAL = 0, 1, 2, 3
TIMER_NAMES = ("radix", "permute", "offsets", "collide", "deposit", "poisson", "field", "push",
               "inject")
EXPORTED = ("pd_create", "pd_set_species", "pd_set_cross_section", "pd_set_heavy_subcycle",
            "pd_set_emission", "pd_set_circuit", "pd_set_split_literal", "pd_set_sputtering",
            "pd_set_weighted", "pd_inject", "pd_inject_weighted", "pd_get_weights",
            "pd_schedule_injection", "pd_step", "pd_synchronize", "pd_get_diagnostics",
            "pd_get_spectrum", "pd_get_count", "pd_get_particles", "pd_get_field",
            "pd_poisson", "pd_poisson_noalloc", "pd_save", "pd_load", "pd_get_timing", "pd_set_timing", "pd_last_error", "pd_destroy",
            "pd_unet_create", "pd_unet_info", "pd_unet_set_weights", "pd_unet_get_weights",
            "pd_unet_forward", "pd_unet_gradient", "pd_unet_add_sample", "pd_unet_train",
            "pd_set_unet", "pd_unet_last_error", "pd_unet_destroy",
            "pd_ensemble_create", "pd_ensemble_step", "pd_ensemble_synchronize",
            "pd_ensemble_last_error", "pd_ensemble_destroy")


class PdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class pd_domain(C.Structure):
    _fields_ = [("nr", C.c_int32), ("nz", C.c_int32), ("R", C.c_double), ("L", C.c_double),
                ("V_cathode", C.c_double), ("dt", C.c_double), ("weight", C.c_double),
                ("seed", C.c_uint64), ("capacity", C.c_int64)]


class pd_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("poisson", C.c_int32), ("enable_di", C.c_int32),
                ("deposit_off", C.c_int32), ("collisions_off", C.c_int32), ("timing", C.c_int32),
                ("stream", C.c_void_p), ("poisson_rtol", C.c_double)]


PD_NSPECIES, PD_NCHANNELS = 8, 10


class pd_diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("n_alive", C.c_int64), ("next_id", C.c_int64),
                ("count", C.c_int64 * PD_NSPECIES), ("events", C.c_int64 * PD_NCHANNELS),
                ("conflicts", C.c_int64),
                ("created", C.c_int64), ("absorbed", (C.c_int64 * PD_NSPECIES) * 3),
                ("injected", C.c_int64 * PD_NSPECIES), ("charge_alive", C.c_int64),
                ("charge_absorbed", C.c_int64), ("charge_injected", C.c_int64),
                ("ke_J", C.c_double * PD_NSPECIES), ("gamma", C.c_double), ("qbar", C.c_double),
                ("particle_steps", C.c_int64), ("poisson_rel_res", C.c_double),
                ("poisson_solves", C.c_int64), ("poisson_iters", C.c_int64),
                ("poisson_refinements", C.c_int64), ("poisson_fallbacks", C.c_int64),
                ("poisson_seconds", C.c_double), ("V_gap", C.c_double),
                ("emitted", C.c_int64 * 2), ("sputtered", C.c_int64),
                ("real", C.c_int64 * PD_NSPECIES)]


_lib = None


def load_library(path=LIB_PATH):
    """Load libpd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libpd.so not built (run __graft_entry__.build()): %s" % path)
    lib = C.CDLL(path)
    P = C.c_void_p
    lib.pd_create.argtypes = [C.POINTER(pd_domain), C.POINTER(pd_opts), C.POINTER(C.c_void_p)]
    lib.pd_set_species.argtypes = [P, C.c_int, P, P]
    lib.pd_set_cross_section.argtypes = [P, C.c_int, C.c_double, C.c_int, C.c_double, P]
    lib.pd_inject.argtypes = [P, C.c_int64] + [P] * 6
    lib.pd_inject_weighted.argtypes = [P, C.c_int64] + [P] * 7
    lib.pd_set_weighted.argtypes = [P, C.c_int32]
    lib.pd_get_weights.argtypes = [P, C.c_int64, P]
    lib.pd_schedule_injection.argtypes = [P, C.c_int, P] + [P] * 6
    lib.pd_step.argtypes = [P, C.c_int]
    lib.pd_synchronize.argtypes = [P]
    lib.pd_get_diagnostics.argtypes = [P, C.POINTER(pd_diag)]
    lib.pd_get_spectrum.argtypes = [P, C.c_int, P]
    lib.pd_get_count.argtypes = [P, C.POINTER(C.c_int64)]
    lib.pd_get_particles.argtypes = [P, C.c_int64] + [P] * 8
    lib.pd_get_field.argtypes = [P, P, P, P, P]
    lib.pd_poisson.argtypes = [P, P, P, C.POINTER(C.c_int32), C.POINTER(C.c_double)]
    lib.pd_poisson_noalloc.argtypes = [P, P, P, P]
    lib.pd_save.argtypes = [P, C.c_char_p]
    lib.pd_set_heavy_subcycle.argtypes = [P, C.c_int32]
    lib.pd_set_emission.argtypes = [P] + [C.c_double] * 5
    lib.pd_set_circuit.argtypes = [P] + [C.c_double] * 3
    lib.pd_set_split_literal.argtypes = [P, C.c_int32]
    lib.pd_set_sputtering.argtypes = [P, C.c_int32]
    lib.pd_load.argtypes = [P, C.c_char_p]
    lib.pd_get_timing.argtypes = [P, P, C.POINTER(C.c_int64), C.c_int]
    lib.pd_set_timing.argtypes = [P, C.c_int]
    lib.pd_last_error.argtypes = [P]
    lib.pd_last_error.restype = C.c_char_p
    lib.pd_unet_create.argtypes = [C.c_int32] * 5 + [C.c_int64, C.POINTER(C.c_void_p)]
    lib.pd_unet_info.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int32)]
    lib.pd_unet_set_weights.argtypes = [P, P]
    lib.pd_unet_get_weights.argtypes = [P, P]
    lib.pd_unet_forward.argtypes = [P, C.c_int32, P, P]
    lib.pd_unet_gradient.argtypes = [P, C.c_int32, P, P, P]
    lib.pd_unet_add_sample.argtypes = [P, P]
    lib.pd_unet_train.argtypes = [P, C.c_int32, C.c_int32, C.c_double, C.c_uint64,
                                  C.POINTER(C.c_double)]
    lib.pd_set_unet.argtypes = [P, P]
    lib.pd_unet_last_error.argtypes = [P]
    lib.pd_unet_last_error.restype = C.c_char_p
    lib.pd_unet_destroy.argtypes = [P]
    lib.pd_unet_destroy.restype = None
    lib.pd_ensemble_create.argtypes = [C.c_int32, P, C.c_int32, C.POINTER(C.c_void_p)]
    lib.pd_ensemble_step.argtypes = [P, C.c_int32]
    lib.pd_ensemble_synchronize.argtypes = [P]
    lib.pd_ensemble_last_error.argtypes = [P]
    lib.pd_ensemble_last_error.restype = C.c_char_p
    lib.pd_ensemble_destroy.argtypes = [P]
    lib.pd_ensemble_destroy.restype = None
    lib.pd_destroy.argtypes = [P]
    lib.pd_destroy.restype = None
    for name in EXPORTED:
        if name not in ("pd_last_error", "pd_destroy", "pd_unet_last_error", "pd_unet_destroy",
                        "pd_ensemble_last_error", "pd_ensemble_destroy"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(ctx, status):
    if status != PD_OK:
        msg = load_library().pd_last_error(ctx)
        raise PdError(status, msg.decode() if msg else "")


# ---- functions with the C names (marshalling only) -------------------------
def pd_create(dom, opts):
    lib = load_library()
    h = C.c_void_p()
    _check(None, lib.pd_create(C.byref(dom), C.byref(opts), C.byref(h)))
    return h


def pd_set_species(ctx, Z, mass):
    Z = np.ascontiguousarray(Z, np.int32)
    m = np.ascontiguousarray(mass, np.float64)
    _check(ctx, load_library().pd_set_species(ctx, len(Z), _ptr(Z), _ptr(m)))


def pd_set_cross_section(ctx, channel, threshold_eV, dsqrtE, sigma):
    s = np.ascontiguousarray(sigma, np.float64)
    _check(ctx, load_library().pd_set_cross_section(ctx, channel, threshold_eV, len(s), dsqrtE,
                                                    _ptr(s)))


def _parts(p):
    return [np.ascontiguousarray(p[k], np.float64) for k in ("r", "z", "vr", "vt", "vz")] + [
        np.ascontiguousarray(p["sp"], np.uint8)]


def pd_inject(ctx, parts):
    a = _parts(parts)
    _check(ctx, load_library().pd_inject(ctx, len(a[0]), *[_ptr(x) for x in a]))


def pd_schedule_injection(ctx, offsets, parts):
    off = np.ascontiguousarray(offsets, np.int64)
    a = _parts(parts)
    _check(ctx, load_library().pd_schedule_injection(ctx, len(off) - 1, _ptr(off),
                                                     *[_ptr(x) for x in a]))


def pd_step(ctx, nsteps=1):
    _check(ctx, load_library().pd_step(ctx, nsteps))


def pd_synchronize(ctx):
    _check(ctx, load_library().pd_synchronize(ctx))


def pd_get_diagnostics(ctx):
    d = pd_diag()
    _check(ctx, load_library().pd_get_diagnostics(ctx, C.byref(d)))
    out = {}
    for name, _ in pd_diag._fields_:
        v = getattr(d, name)
        out[name] = v if isinstance(v, (int, float)) else np.array(
            [list(x) if not isinstance(x, (int, float)) else x for x in v])
    return out


def pd_get_spectrum(ctx, tag):
    out = np.zeros(66, np.int64)
    _check(ctx, load_library().pd_get_spectrum(ctx, tag, _ptr(out)))
    return out


def pd_get_count(ctx):
    n = C.c_int64()
    _check(ctx, load_library().pd_get_count(ctx, C.byref(n)))
    return n.value


def pd_get_particles(ctx):
    n = pd_get_count(ctx)
    out = {k: np.zeros(n, np.float64) for k in ("r", "z", "vr", "vt", "vz")}
    out["sp"] = np.zeros(n, np.uint8)
    out["id"] = np.zeros(n, np.uint32)
    out["key"] = np.zeros(n, np.uint32)
    _check(ctx, load_library().pd_get_particles(
        ctx, n, *[_ptr(out[k]) for k in ("r", "z", "vr", "vt", "vz", "sp", "id", "key")]))
    return out


def pd_get_field(ctx, nr, nz):
    nn = (nr + 1) * (nz + 1)
    phi, Er, Ez = (np.zeros(nn) for _ in range(3))
    Q = np.zeros(nn, np.int64)
    _check(ctx, load_library().pd_get_field(ctx, _ptr(phi), _ptr(Er), _ptr(Ez), _ptr(Q)))
    shp = (nz + 1, nr + 1)
    return {"phi": phi.reshape(shp), "Er": Er.reshape(shp), "Ez": Ez.reshape(shp),
            "Q": Q.reshape(shp)}


def pd_poisson(ctx, Q, nr, nz):
    """Solve for node charges Q; returns (phi, CG iterations, relative residual)."""
    q = np.ascontiguousarray(Q, np.int64).reshape(-1)
    if q.size != (nr + 1) * (nz + 1):
        raise ValueError("Q has %d values, the grid %d nodes" % (q.size, (nr + 1) * (nz + 1)))
    phi = np.zeros(q.size)
    it = C.c_int32()
    rel = C.c_double()
    _check(ctx, load_library().pd_poisson(ctx, _ptr(q), _ptr(phi), C.byref(it), C.byref(rel)))
    return phi.reshape(nz + 1, nr + 1), it.value, rel.value


def pd_poisson_noalloc(ctx, q_dev, phi_dev, stream=None):
    """Direct solve for a node charge in device memory (q_dev, phi_dev:
    device addresses as integers); enqueues and returns (no synchronisation)."""
    _check(ctx, load_library().pd_poisson_noalloc(ctx, C.c_void_p(q_dev), C.c_void_p(phi_dev),
                                                  C.c_void_p(stream)))


def pd_set_heavy_subcycle(ctx, every):
    _check(ctx, load_library().pd_set_heavy_subcycle(ctx, int(every)))


def pd_set_emission(ctx, beta, r_tip, phi_w, neutral_ratio, T):
    _check(ctx, load_library().pd_set_emission(ctx, beta, r_tip, phi_w, neutral_ratio, T))


def pd_set_circuit(ctx, V0, R, C_farad):
    _check(ctx, load_library().pd_set_circuit(ctx, V0, R, C_farad))


def pd_set_split_literal(ctx, on):
    _check(ctx, load_library().pd_set_split_literal(ctx, 1 if on else 0))


def pd_set_sputtering(ctx, on):
    _check(ctx, load_library().pd_set_sputtering(ctx, 1 if on else 0))


def pd_set_weighted(ctx, on):
    _check(ctx, load_library().pd_set_weighted(ctx, 1 if on else 0))


def pd_inject_weighted(ctx, parts, mu):
    a = _parts(parts)
    m = np.ascontiguousarray(mu, dtype=np.uint16)
    if len(m) != len(a[0]):
        raise ValueError("one multiplicity per particle")
    _check(ctx, load_library().pd_inject_weighted(ctx, len(a[0]), *[_ptr(x) for x in a],
                                                  _ptr(m)))


def pd_get_weights(ctx):
    n = pd_get_count(ctx)
    out = np.zeros(n, np.uint16)
    _check(ctx, load_library().pd_get_weights(ctx, n, _ptr(out)))
    return out


def pd_save(ctx, path):
    _check(ctx, load_library().pd_save(ctx, os.fsencode(path)))


def pd_load(ctx, path):
    _check(ctx, load_library().pd_load(ctx, os.fsencode(path)))


def _check_net(net, status):
    if status != PD_OK:
        msg = load_library().pd_unet_last_error(net)
        raise PdError(status, msg.decode() if msg else "")


def pd_unet_create(nr, nz, levels=4, base=16, batch=4, dataset_capacity=0):
    h = C.c_void_p()
    _check_net(None, load_library().pd_unet_create(nr, nz, levels, base, batch,
                                                   int(dataset_capacity), C.byref(h)))
    return h


def pd_unet_info(net):
    n, H, W = C.c_int64(), C.c_int32(), C.c_int32()
    _check_net(net, load_library().pd_unet_info(net, C.byref(n), C.byref(H), C.byref(W)))
    return n.value, H.value, W.value


def pd_unet_set_weights(net, w):
    w = np.ascontiguousarray(w, np.float32)
    _check_net(net, load_library().pd_unet_set_weights(net, _ptr(w)))


def pd_unet_get_weights(net):
    n, _, _ = pd_unet_info(net)
    w = np.zeros(n, np.float32)
    _check_net(net, load_library().pd_unet_get_weights(net, _ptr(w)))
    return w


def pd_unet_forward(net, x):
    x = np.ascontiguousarray(x, np.float32)
    out = np.zeros((x.shape[0], x.shape[2], x.shape[3]), np.float32)
    _check_net(net, load_library().pd_unet_forward(net, x.shape[0], _ptr(x), _ptr(out)))
    return out


def pd_unet_gradient(net, x, dout):
    x = np.ascontiguousarray(x, np.float32)
    d = np.ascontiguousarray(dout, np.float32)
    n, _, _ = pd_unet_info(net)
    dw = np.zeros(n, np.float32)
    _check_net(net, load_library().pd_unet_gradient(net, x.shape[0], _ptr(x), _ptr(d), _ptr(dw)))
    return dw


def pd_unet_add_sample(net, ctx):
    _check_net(net, load_library().pd_unet_add_sample(net, ctx))


def pd_unet_train(net, epochs, batch, lr, seed=1):
    loss = C.c_double()
    _check_net(net, load_library().pd_unet_train(net, epochs, batch, lr, seed, C.byref(loss)))
    return loss.value


def pd_set_unet(ctx, net):
    _check(ctx, load_library().pd_set_unet(ctx, net))


def pd_unet_last_error(net):
    msg = load_library().pd_unet_last_error(net)
    return msg.decode() if msg else ""


def pd_unet_destroy(net):
    if net:
        load_library().pd_unet_destroy(net)


def _check_ens(ens, status):
    if status != PD_OK:
        msg = load_library().pd_ensemble_last_error(ens)
        raise PdError(status, msg.decode() if msg else "")


def pd_ensemble_create(ctxs, nstreams=4):
    arr = (C.c_void_p * len(ctxs))(*[c.value if isinstance(c, C.c_void_p) else c for c in ctxs])
    h = C.c_void_p()
    _check_ens(None, load_library().pd_ensemble_create(len(ctxs), arr, nstreams, C.byref(h)))
    return h


def pd_ensemble_step(ens, nsteps):
    _check_ens(ens, load_library().pd_ensemble_step(ens, nsteps))


def pd_ensemble_synchronize(ens):
    _check_ens(ens, load_library().pd_ensemble_synchronize(ens))


def pd_ensemble_last_error(ens):
    msg = load_library().pd_ensemble_last_error(ens)
    return msg.decode() if msg else ""


def pd_ensemble_destroy(ens):
    if ens:
        load_library().pd_ensemble_destroy(ens)


def pd_get_timing(ctx, reset=False):
    ms = np.zeros(len(TIMER_NAMES))
    steps = C.c_int64()
    _check(ctx, load_library().pd_get_timing(ctx, _ptr(ms), C.byref(steps), int(reset)))
    return dict(zip(TIMER_NAMES, ms.tolist())), steps.value


def pd_set_timing(ctx, on):
    _check(ctx, load_library().pd_set_timing(ctx, int(bool(on))))


def pd_last_error(ctx):
    msg = load_library().pd_last_error(ctx)
    return msg.decode() if msg else ""


def pd_destroy(ctx):
    if ctx:
        load_library().pd_destroy(ctx)


# ---- convenience wrapper ----------------------------------------------------
class Simulation:
    """One context: the domain of a workload config plus species and tables."""

    def __init__(self, cfg, capacity, tables, species, enable_di=None, deposit_off=False,
                 collisions_off=False, timing=False, stream=None, poisson=PD_POISSON_DIRECT64,
                 poisson_rtol=0.0, precision=PD_FP64_DET):
        dom = pd_domain(cfg.nr, cfg.nz, cfg.R, cfg.L, cfg.V, cfg.dt, cfg.weight, cfg.seed,
                        int(capacity))
        di = cfg.enable_di if enable_di is None else enable_di
        opts = pd_opts(precision, poisson, int(di), int(deposit_off), int(collisions_off),
                       int(timing), stream, float(poisson_rtol))
        self.cfg = cfg
        self.h = pd_create(dom, opts)
        pd_set_species(self.h, *species)
        for ch, thr, dsq, sig in tables:
            pd_set_cross_section(self.h, ch, thr, dsq, sig)

    def inject(self, parts, mult=None):
        if mult is None:
            pd_inject(self.h, parts)
        else:
            pd_inject_weighted(self.h, parts, mult)

    def set_weighted(self, on=True):
        pd_set_weighted(self.h, on)

    def weights(self):
        return pd_get_weights(self.h)

    def schedule_injection(self, offsets, parts):
        pd_schedule_injection(self.h, offsets, parts)

    def step(self, n=1):
        pd_step(self.h, n)

    def synchronize(self):
        pd_synchronize(self.h)

    def diag(self):
        return pd_get_diagnostics(self.h)

    def set_heavy_subcycle(self, every):
        pd_set_heavy_subcycle(self.h, every)

    def set_emission(self, beta, r_tip, phi_w, neutral_ratio, T):
        pd_set_emission(self.h, beta, r_tip, phi_w, neutral_ratio, T)

    def set_circuit(self, V0, R, C_farad):
        pd_set_circuit(self.h, V0, R, C_farad)

    def set_split_literal(self, on):
        pd_set_split_literal(self.h, on)

    def set_sputtering(self, on):
        pd_set_sputtering(self.h, on)

    def save(self, path):
        pd_save(self.h, path)

    def load(self, path):
        pd_load(self.h, path)

    def spectrum(self, tag):
        return pd_get_spectrum(self.h, tag)

    def count(self):
        return pd_get_count(self.h)

    def particles(self):
        return pd_get_particles(self.h)

    def field(self):
        return pd_get_field(self.h, self.cfg.nr, self.cfg.nz)

    def poisson(self, Q):
        return pd_poisson(self.h, Q, self.cfg.nr, self.cfg.nz)

    def timing(self, reset=False):
        return pd_get_timing(self.h, reset)

    def set_timing(self, on):
        pd_set_timing(self.h, on)

    def close(self):
        if getattr(self, "h", None):
            pd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: the module's functions may be gone
            pass
