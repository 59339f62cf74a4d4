"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle.

This package draws random inputs only; it contains none of the spectrum
model's arithmetic (no line strengths, widths, profiles, transfer or
response).  Both the HIP path and the oracle consume what it returns.
"""
from .workloads import (  # noqa: F401
    LineList, Atmosphere, Response, Workload, ServingRequest, make_config,
    eslog_grid, serving_pool, serving_requests, serving_atmosphere, hmc_walk, CONFIG_SEEDS,
)
