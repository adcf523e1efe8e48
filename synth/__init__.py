"""Seeded synthetic inputs shared by the oracle-based tests and the GPU path.

This package draws random fields only; it holds none of the estimator's
arithmetic (no shells, no triangle sums, no normalisation of B).
"""
from .fields import (PowerLaw, batch_field, batch_members, gaussian_field, quadratic_ng_field,
                     workload_field, WORKLOADS)

__all__ = ["PowerLaw", "gaussian_field", "quadratic_ng_field", "workload_field", "WORKLOADS", "batch_members",
           "batch_field"]
