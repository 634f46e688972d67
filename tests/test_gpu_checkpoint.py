"""GPU checks of the checkpoint (pd_save / pd_load) through the C-ABI:

  - resume: 200 steps of the 32x64 workload equal, bit for bit, 100 steps +
    pd_save + pd_load into a fresh context + 100 steps (every particle field,
    node charge, potential, field, counter and spectrum), in the FP64 form
    with the direct solve, with MG-PCG (whose adaptive iteration count is part
    of the state) and in the FP32 form; the resumed run also equals the oracle
    stepped 200 times (FP64, direct);
  - file errors: a truncated file, a wrong magic, a file of another domain and
    a missing file return PD_EINVAL and leave the loading context as it was.
"""
import os

import numpy as np
import pytest

from conftest import make_oracle
from gpu_common import assert_same_state, gpu_sim, log
from paper_2109_00214_amd import workload as W

pytestmark = pytest.mark.gpu


def _same_everything(a, b, where):
    pa, pb = a.particles(), b.particles()
    for k in pa:
        x, y = pa[k], pb[k]
        same = np.array_equal(x.view(np.uint64 if x.dtype.itemsize == 8 else np.uint32), y.view(
            np.uint64 if y.dtype.itemsize == 8 else np.uint32)) if x.dtype.kind == "f" else \
            np.array_equal(x, y)
        assert same, "%s: particle field %s differs" % (where, k)
    fa, fb = a.field(), b.field()
    for k in ("Q", "phi", "Er", "Ez"):
        assert np.array_equal(fa[k].view(np.uint64), fb[k].view(np.uint64)), (where, k)
    da, db = a.diag(), b.diag()
    for k in ("step", "n_alive", "next_id", "count", "events", "conflicts", "created", "absorbed",
              "injected", "charge_alive", "charge_absorbed", "charge_injected", "particle_steps",
              "poisson_iters", "poisson_refinements", "poisson_fallbacks"):
        assert np.array_equal(np.asarray(da[k]), np.asarray(db[k])), (where, k)
    for tag in range(3):
        assert np.array_equal(a.spectrum(tag), b.spectrum(tag)), (where, tag)


@pytest.mark.parametrize("form", ["direct", "mgpcg", "fp32"])
def test_resume_after_save_and_load_is_bit_exact(form, tmp_path):
    from paper_2109_00214_amd import pd
    log("case: checkpoint resume, tiny workload, %s" % form)
    cfg = W.config("tiny")
    kw = {"direct": {}, "mgpcg": {"poisson": pd.PD_POISSON_MGPCG},
          "fp32": {"precision": pd.PD_FP32_MIXED}}[form]
    parts = W.initial_population(cfg)
    off, inj = W.injection_schedule(cfg, 200)
    cap = 200_000
    ref = gpu_sim(cfg, cap, **kw)
    ref.inject(parts)
    ref.schedule_injection(off, inj)
    ref.step(100)
    path = str(tmp_path / "state.pd")
    ref.save(path)
    ref.step(100)
    fresh = gpu_sim(cfg, cap, **kw)
    fresh.load(path)
    fresh.step(100)
    _same_everything(ref, fresh, "resumed %s" % form)
    if form == "direct":
        o = make_oracle(cfg)
        o.inject(parts)
        o.schedule_injection(off, inj)
        o.step(200)
        assert_same_state(fresh, o, "resumed run against the oracle")
    ref.close()
    fresh.close()


def test_load_errors_leave_the_context_unchanged(tmp_path):
    from paper_2109_00214_amd import pd
    log("case: checkpoint file errors")
    cfg = W.config("tiny", n_init=5000)
    src = gpu_sim(cfg, 40_000)
    src.inject(W.initial_population(cfg))
    src.step(3)
    good = str(tmp_path / "good.pd")
    src.save(good)
    blob = open(good, "rb").read()
    # the context that receives the bad files already holds a state
    dst = gpu_sim(cfg, 40_000)
    dst.inject(W.initial_population(cfg, n=2000))
    dst.step(2)
    before = dst.particles()
    other = W.config("tiny", nr=16, nz=32, n_init=100)
    osim = gpu_sim(other, 4096)
    osim.inject(W.initial_population(other))
    wrong_domain = str(tmp_path / "other.pd")
    osim.save(wrong_domain)
    bad = {"truncated": blob[: len(blob) // 2], "magic": b"XXXXXXXX" + blob[8:],
           "tail": blob[:-8] + b"XXXXXXXX", "extra": blob + b"\0"}
    cases = []
    for name, data in bad.items():
        p = str(tmp_path / (name + ".pd"))
        open(p, "wb").write(data)
        cases.append(p)
    cases += [wrong_domain, str(tmp_path / "missing.pd")]
    for p in cases:
        with pytest.raises(pd.PdError) as ei:
            dst.load(p)
        assert ei.value.status == pd.PD_EINVAL, (os.path.basename(p), ei.value)
        after = dst.particles()
        for k in before:
            assert np.array_equal(before[k], after[k]), (os.path.basename(p), k)
    # and the good file still loads
    dst.load(good)
    assert dst.count() == src.count()
    for s in (src, dst, osim):
        s.close()
