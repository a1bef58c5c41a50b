"""MI355X-native plane-wave Gamma-point Hartree-Fock exact exchange.

The computation runs in hand-written HIP kernels for gfx950 behind the C ABI
of ``include/hfx.h`` (``libhfx.so``); :mod:`paper_2309_00651_amd.hfx` is the
thin ctypes binding.  Build with ``python -m paper_2309_00651_amd.build``.
"""
from .hfx import (ERFC, FP32, FP64, TRUNCATED, ExchangeEnergy, HfxError, Plan,  # noqa: F401
                  SystemSpec, apply_exchange, exchange_energy, exchange_matrix,
                  load_library, orthonormalize)
