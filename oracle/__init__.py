"""FP64 CPU oracle for plane-wave Gamma-point exact exchange.

Test infrastructure only: imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py.  The HIP library never imports this package.
"""
from .hfx_oracle import *  # noqa: F401,F403
from .hfx_oracle import __all__  # noqa: F401
