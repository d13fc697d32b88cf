"""Seeded synthetic catalogs shared by the oracle, the tests and the benchmark.

This package only *generates inputs*: lognormal galaxy catalogs, uniform random
catalogs, fixed-amplitude Gaussian meshes and tiny hand-made catalogs.  It holds
none of the estimator arithmetic (no painting, no multipole weighting, no
binning, no bispectrum), so both the FP64 oracle and the GPU library can consume
its output without sharing any of the method's code.

Positions are quantised to 3 x uint32 fixed point, p = floor(x / L * 2**32),
stored structure-of-arrays as a C-contiguous ``(3, n)`` uint32 array.
"""

from .lognormal import (
    CONFIGS,
    ConfigSpec,
    config_spec,
    fixed_amplitude_mesh,
    lognormal_catalog,
    mock_sizes_c4,
    poisson_catalog,
    random_catalog,
    tiny_catalog,
    observer_position,
    field_power,
)

__all__ = [
    "CONFIGS",
    "ConfigSpec",
    "config_spec",
    "fixed_amplitude_mesh",
    "lognormal_catalog",
    "mock_sizes_c4",
    "poisson_catalog",
    "random_catalog",
    "tiny_catalog",
    "observer_position",
    "field_power",
]
