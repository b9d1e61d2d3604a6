"""Seeded synthetic inputs shared by the tests, the oracle checks and the benchmark.

This package holds none of the method's arithmetic: it draws random numbers,
evaluates smooth test functions on grids and returns plain numpy arrays.
Neither the oracle nor the GPU library is imported here.
"""
from .inputs import *  # noqa: F401,F403
