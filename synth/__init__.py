"""Seeded synthetic inputs for the local block-sparse multiply.

This module only draws random patterns and values; it holds none of the
multiply's arithmetic.  The GPU library's tests, the benchmark and the CPU
reference all take their inputs from here.
"""
from .blocks import *  # noqa: F401,F403
