"""brng: MI355X-native varying-parameter random number generation.

A HIP (gfx950) implementation of the buffered-RNG method of Mahani &
Sharabiani (arXiv 1412.4825): Philox4x32-10 fills pools of standard uniform,
Gaussian and exponential deviates in HBM; many independent chains consume
them one deviate at a time with per-step parameters.  The C interface is in
include/brng.h; ``binding`` exposes it under the same names.
"""
from . import workloads  # noqa: F401

__all__ = ["binding", "workloads"]
