"""Seeded synthetic inputs for the convolution-product expansion.

This package only *describes* operators and draws inputs: kernels / TVIRs,
B-spline and tile windows, impulse responses sampled from a TVIR, and the
signals.  It holds none of the expansion's arithmetic (no convolution, no
transform, no sum over terms); both the FP64 oracle and the GPU path consume
what it produces.
"""
from .gen import *  # noqa: F401,F403
