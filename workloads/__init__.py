"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package holds input generation only (random numbers, inverse-CDF sampling of the
initial density, the workload catalogue).  It contains none of the particle-in-cell
step's arithmetic, and it imports neither the oracle nor the GPU package.
"""
from .generators import (  # noqa: F401
    uniforms, normals, sample_density, Workload, landau, landau_2v, two_stream, weibel,
    batched_landau, adjoint_two_stream, catalogue, by_name,
)
