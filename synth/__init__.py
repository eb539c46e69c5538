"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package draws random numbers and describes workloads (mesh sizes, cuts,
Robin coefficients, density anomalies). It holds none of the solver's
arithmetic: no finite-element matrices, no Schwarz step, no Krylov step.
"""
from .generators import (  # noqa: F401
    blob_params,
    blobs_density,
    crater_density,
    uniform_density,
    random_widths,
    element_centroids,
)
from .workloads import Workload, workload, WORKLOADS  # noqa: F401
