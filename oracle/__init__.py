"""FP64 CPU oracle of multilevel summation for r^-6 dispersion.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``, never by the library.  It shares no
code with the HIP path.
"""
from . import exact, lattice, mls  # noqa: F401
from .mls import mls as evaluate  # noqa: F401
