"""Seeded synthetic regression problems shared by the tests, the benchmark and
the oracle.  This module generates inputs only: it holds none of the method's
arithmetic (no sketch, no solver, no reference result).
"""
from .generators import (  # noqa: F401
    WORKLOADS,
    batched_shapes,
    Problem,
    fingerprint,
    make_problem,
    make_batched,
    paper_problem,
    sketch_seed,
)
