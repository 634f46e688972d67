"""GPU check of pd_poisson_noalloc, the entry point that allocates nothing
(its intermediate arrays live in the library's fixed per-GPU scratch): through
the C-ABI, the potential it writes into caller device memory equals, bit for
bit, the one pd_poisson returns for the same node charge (the same
fixed-order direct solve), and the oracle's.  Two calls in a row, the second
on a smaller grid; then the refusals (a grid beyond the scratch, a context
without the fixed-order solve) leave the caller's buffer untouched."""
import numpy as np
import pytest

from conftest import make_oracle
from gpu_common import gpu_sim, log
from paper_2109_00214_amd import workload as W

pytestmark = pytest.mark.gpu


class _Dev:
    """Device buffers from the HIP runtime the library itself runs on (test
    infrastructure: the caller's memory that the entry point writes into)."""

    def __init__(self):
        import ctypes as C
        from paper_2109_00214_amd import pd
        pd.load_library()
        self.C = C
        self.hip = C.CDLL("libamdhip64.so.7")  # the copy the library has loaded

    def alloc(self, nbytes):
        p = self.C.c_void_p()
        assert self.hip.hipMalloc(self.C.byref(p), self.C.c_size_t(nbytes)) == 0
        return p.value

    def put(self, dst, a):
        a = np.ascontiguousarray(a)
        assert self.hip.hipMemcpy(self.C.c_void_p(dst), a.ctypes.data_as(self.C.c_void_p),
                                  self.C.c_size_t(a.nbytes), 1) == 0  # host to device

    def get(self, src, a):
        assert self.hip.hipMemcpy(a.ctypes.data_as(self.C.c_void_p), self.C.c_void_p(src),
                                  self.C.c_size_t(a.nbytes), 2) == 0  # device to host
        return a

    def sync(self):
        assert self.hip.hipDeviceSynchronize() == 0

    def free(self, p):
        assert self.hip.hipFree(self.C.c_void_p(p)) == 0


def _charge(cfg, n):
    o = make_oracle(cfg, collisions_off=True)
    o.inject(W.initial_population(cfg, n=n))
    for st in ("sort", "collide", "deposit"):
        o.stage(st)
    return o, o.field()["Q"].copy()


def test_noalloc_solve_equals_pd_poisson_twice_then_smaller():
    from paper_2109_00214_amd import pd
    dev = _Dev()
    for (nr, nz), n in (((64, 128), 60_000), ((32, 64), 20_000)):
        log("case: pd_poisson_noalloc, %dx%d, %d particles" % (nr, nz, n))
        cfg = W.config("tiny", nr=nr, nz=nz)
        o, Q = _charge(cfg, n)
        g = gpu_sim(cfg, 1024)
        ref, it, _ = g.poisson(Q)
        assert it == 0
        q_dev, phi_dev = dev.alloc(8 * Q.size), dev.alloc(8 * Q.size)
        dev.put(q_dev, Q.reshape(-1).astype(np.int64))
        dev.put(phi_dev, np.full(Q.size, np.nan))
        dev.sync()
        pd.pd_poisson_noalloc(g.h, q_dev, phi_dev, None)
        g.synchronize()
        phi = dev.get(phi_dev, np.empty(Q.size)).reshape(ref.shape)
        dev.free(q_dev)
        dev.free(phi_dev)
        bad = np.nonzero(phi.view(np.uint64) != ref.view(np.uint64))
        assert bad[0].size == 0, "first differing node (row, column): %s" % (
            [int(bad[0][0]), int(bad[1][0])],)
        o.stage("poisson")
        assert np.array_equal(phi.view(np.uint64), o.field()["phi"].view(np.uint64))
        g.close()


def test_noalloc_refusals_leave_output_untouched():
    from paper_2109_00214_amd import pd
    log("case: pd_poisson_noalloc refusals")
    dev = _Dev()
    for (nr, nz), mode in (((1023, 512), pd.PD_POISSON_DIRECT64),
                           ((32, 64), pd.PD_POISSON_SPECTRAL)):
        cfg = W.config("tiny", nr=nr, nz=nz)
        g = gpu_sim(cfg, 1024, poisson=mode)
        nn = (nr + 1) * (nz + 1)
        q_dev, phi_dev = dev.alloc(8 * nn), dev.alloc(8 * nn)
        dev.put(q_dev, np.zeros(nn, np.int64))
        dev.put(phi_dev, np.full(nn, 7.0))
        dev.sync()
        with pytest.raises(pd.PdError) as ei:
            pd.pd_poisson_noalloc(g.h, q_dev, phi_dev, None)
        assert ei.value.status == pd.PD_EINVAL
        dev.sync()
        assert np.all(dev.get(phi_dev, np.empty(nn)) == 7.0)
        dev.free(q_dev)
        dev.free(phi_dev)
        g.close()
