"""MI355X (gfx950) r-z electrostatic PIC-DSMC step with the direct
double-ionization channel of arXiv 2109.00214.

``pd`` is the ctypes binding of the HIP library (``libpd.so``, built by
``build.build_library``); ``workload`` draws the seeded synthetic inputs.
"""
from . import workload  # noqa: F401
