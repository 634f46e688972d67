"""Plain FP64 CPU oracle of the r-z PIC-DSMC step (arXiv 2109.00214, Sec. 2).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``; never by the product package.
The C source is ``oracle/pd_oracle.c``; this module is a thin ctypes wrapper.
"""
from .oracle import Oracle, build_oracle, oracle_lib, philox4x32_10  # noqa: F401
