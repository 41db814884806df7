"""Seeded synthetic inputs (graph realizations with an embedded target), shared by tests and benchmarks.

Holds none of the method's arithmetic: only random graph construction and CSR assembly.
"""
from . import graphs, configs  # noqa: F401
