"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

Holds mesh generators, seeded fields and the problem definitions.  It holds
none of the method's arithmetic (no shape functions, volumes, areas, time
steps or updates), so the oracle and the GPU path stay independent.
"""
from . import fields, mesh, problems  # noqa: F401
