"""FP64 CPU oracle of the compact 6th/8th-order gas-kinetic scheme.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The product path (the HIP library and its
binding) never imports it.
"""
from .oracle import *  # noqa: F401,F403
