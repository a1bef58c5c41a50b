"""Seeded synthetic inputs (orbital generators and named workloads).

Shared by the oracle tests, the HIP tests and the benchmark; holds no exchange
arithmetic.
"""
from . import configs, generate  # noqa: F401
