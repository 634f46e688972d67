"""CPU checks of the C-ABI library: it loads and exports every entry point
that include/pd.h declares (no compute calls: no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pd_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def libpath():
    from paper_2109_00214_amd import build
    if not os.path.exists(build.LIB):
        build.build_library()
    return build.LIB


def test_library_exports_every_declared_symbol(libpath):
    names = _declared()
    assert "pd_step" in names and "pd_create" in names
    lib = ctypes.CDLL(libpath)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header(libpath):
    from paper_2109_00214_amd import pd
    assert sorted(pd.EXPORTED) == _declared()
    for n in pd.EXPORTED:
        assert callable(getattr(pd, n))


def test_struct_layouts_match_header():
    """The ctypes mirrors have the sizes the C compiler gives the structs."""
    import subprocess
    import tempfile
    from paper_2109_00214_amd import pd
    prog = r'''
#include <stdio.h>
#include <stddef.h>
#include "pd.h"
int main(void){ printf("%zu %zu %zu %zu %zu %zu %zu\n", sizeof(pd_domain), sizeof(pd_opts), sizeof(pd_diag),
  offsetof(pd_diag, particle_steps), offsetof(pd_opts, poisson_rtol),
  offsetof(pd_diag, poisson_fallbacks), offsetof(pd_diag, poisson_seconds)); return 0; }
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(prog)
        exe = os.path.join(d, "t")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe]).decode().split()
    assert int(out[0]) == ctypes.sizeof(pd.pd_domain)
    assert int(out[1]) == ctypes.sizeof(pd.pd_opts)
    assert int(out[2]) == ctypes.sizeof(pd.pd_diag)
    assert int(out[3]) == pd.pd_diag.particle_steps.offset
    assert int(out[4]) == pd.pd_opts.poisson_rtol.offset
    assert int(out[5]) == pd.pd_diag.poisson_fallbacks.offset
    assert int(out[6]) == pd.pd_diag.poisson_seconds.offset


def test_missing_library_fails_loudly(tmp_path):
    from paper_2109_00214_amd import pd
    with pytest.raises(ImportError):
        pd._lib_saved = pd._lib
        pd._lib = None
        try:
            pd.load_library(str(tmp_path / "nope.so"))
        finally:
            pd._lib = pd._lib_saved
