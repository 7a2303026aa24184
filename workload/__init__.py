"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle's callers."""
from . import synth, configs  # noqa: F401
