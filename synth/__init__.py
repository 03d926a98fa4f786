"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds no arithmetic of the loop-estimation method itself: it only
draws the gauge configurations (the input data of every solve) and names the
workload configurations.  Z(4) noise is *not* drawn here: it is part of the
method and each side implements the same published counter-based generator on
its own.
"""
from .links import random_su3_links, unit_links
from .configs import CONFIGS, get_config

__all__ = ["random_su3_links", "unit_links", "CONFIGS", "get_config"]
