"""ORACLE — test infrastructure only (tests, the smoke check and the benchmark's CPU-baseline leg).

Plain CPU implementation of DOPE (Algorithm 1 with Theorem 1's block parameters) in exact integer fixed
point, used to check the GPU path.  The product library never imports it."""
from . import dope  # noqa: F401
