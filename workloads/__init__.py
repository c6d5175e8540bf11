"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark."""
from .gen import Csr, generate, CONFIGS, equal_bounds, from_arrays  # noqa: F401
