"""MI355X-native FFT-based binned 3D bispectrum estimator (arXiv:2107.14564).

`Plan` wraps one plan of the HIP library (include/bispec.h); `bispectrum`
is its differentiable entry point; `BatchPlan` runs many configurations
(realisations) back to back, replayed from one captured HIP graph.  PyTorch supplies device memory and the
current HIP stream only.
"""
from __future__ import annotations

from ._abi import (BispecError, FLAG_AUTOTUNE, FLAG_GRAD, FLAG_NO_WORKSPACE, FLAG_ONE_GRID, FLAG_STAGE_TIMING, PREC_FP32, PREC_SPLITBF16, TRI_ALL, TRI_K1SET,
                   TRI_LIST, TRI_MUT_GRID, bispec_contraction_tiles, bispec_estimator_grid, bispec_grid_classes, bispec_query_quads,
                   bispec_query_triangles, bispec_shell_stats,
                   bispec_workspace_bytes, make_config)
from .plan import BatchPlan, Plan, bispectrum

__all__ = ["Plan", "BatchPlan", "bispectrum", "BispecError", "make_config", "bispec_query_triangles", "bispec_shell_stats",
           "bispec_workspace_bytes", "bispec_estimator_grid", "TRI_ALL", "TRI_K1SET", "TRI_MUT_GRID", "TRI_LIST", "PREC_SPLITBF16",
           "PREC_FP32", "FLAG_GRAD", "FLAG_STAGE_TIMING", "FLAG_AUTOTUNE", "FLAG_NO_WORKSPACE", "FLAG_ONE_GRID",
           "bispec_grid_classes", "bispec_contraction_tiles", "bispec_query_quads"]
