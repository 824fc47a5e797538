"""Seeded synthetic inputs (configurations, rigs, rendered pairs and ground truth).

Shared by the tests, the benchmark and the smoke check; holds none of the
method's arithmetic.
"""
from . import configs, scene  # noqa: F401
