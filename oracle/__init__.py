"""CPU oracle for the trajectory nearest-neighbour search.

TEST INFRASTRUCTURE ONLY.  Tests, the smoke check and the benchmark's CPU
baseline use it; the GPU library never imports, links or calls it, and it
imports nothing from the GPU library.
"""
from .oracle import *  # noqa: F401,F403
