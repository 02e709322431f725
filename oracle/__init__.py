"""FP64 CPU oracle for FMCW SAR back-projection (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may import this package.  The product path never does.
"""
from .sar_oracle import *  # noqa: F401,F403
from .sar_oracle import __all__  # noqa: F401
