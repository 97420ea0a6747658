"""Seeded synthetic inputs for adaptive k-NN tests and benchmarks.

This module only draws data (numpy PCG64, fixed seeds).  It holds none of
the method's arithmetic, and both the oracle-side tests and the GPU side
use it.
"""
from .generators import *  # noqa: F401,F403
