"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

Holds lattice/velocity generators and the potential tables; none of the EAM
energy, force or integration arithmetic.
"""
from . import configs, potential  # noqa: F401
