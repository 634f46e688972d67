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


def _charge(cfg, n):
    o = make_oracle(cfg, collisions_off=True)
    o.inject(W.initial_population(cfg, n=n))
    for st in ("sort", "collide", "deposit"):
        o.stage(st)
    return o, o.field()["Q"].copy()


def test_noalloc_solve_equals_pd_poisson_twice_then_smaller():
    import torch

    from paper_2109_00214_amd import pd
    for (nr, nz), n in (((64, 128), 60_000), ((32, 64), 20_000)):
        log("case: pd_poisson_noalloc, %dx%d, %d particles" % (nr, nz, n))
        cfg = W.config("tiny", nr=nr, nz=nz)
        o, Q = _charge(cfg, n)
        g = gpu_sim(cfg, 1024)
        ref, it, _ = g.poisson(Q)
        assert it == 0
        q_dev = torch.from_numpy(np.ascontiguousarray(Q.reshape(-1))).to("cuda")
        phi_dev = torch.full((Q.size,), float("nan"), dtype=torch.float64, device="cuda")
        stream = torch.cuda.current_stream()
        torch.cuda.synchronize()
        pd.pd_poisson_noalloc(g.h, q_dev.data_ptr(), phi_dev.data_ptr(), stream.cuda_stream)
        stream.synchronize()
        phi = phi_dev.cpu().numpy().reshape(ref.shape)
        bad = np.nonzero(phi.view(np.uint64) != ref.view(np.uint64))
        assert bad[0].size == 0, "first differing node (row, column): %s" % (
            [int(bad[0][0]), int(bad[1][0])],)
        o.stage("poisson")
        assert np.array_equal(phi.view(np.uint64), o.field()["phi"].view(np.uint64))
        g.close()


def test_noalloc_refusals_leave_output_untouched():
    import torch

    from paper_2109_00214_amd import pd
    log("case: pd_poisson_noalloc refusals")
    for (nr, nz), mode in (((1023, 512), pd.PD_POISSON_DIRECT64),
                           ((32, 64), pd.PD_POISSON_SPECTRAL)):
        cfg = W.config("tiny", nr=nr, nz=nz)
        g = gpu_sim(cfg, 1024, poisson=mode)
        nn = (nr + 1) * (nz + 1)
        q_dev = torch.zeros(nn, dtype=torch.int64, device="cuda")
        phi_dev = torch.full((nn,), 7.0, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        with pytest.raises(pd.PdError) as ei:
            pd.pd_poisson_noalloc(g.h, q_dev.data_ptr(), phi_dev.data_ptr(), None)
        assert ei.value.status == pd.PD_EINVAL
        torch.cuda.synchronize()
        assert bool(torch.all(phi_dev == 7.0))
        g.close()
