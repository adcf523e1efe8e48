"""Helpers shared by the GPU parity tests: seeded inputs, the GPU call through
the C ABI and the error metrics every result is reported with."""
import sys

import numpy as np


def gpu_ok():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_gpu(delta64):
    import torch
    d32 = np.ascontiguousarray(delta64, dtype=np.float32)
    return torch.from_numpy(d32).cuda(), d32.astype(np.float64)


def metrics(b, ref, s_abs=None):
    """e_norm = |b - ref|_2 / |ref|_2, e_cond = max |b - ref| / S with S the
    oracle's sum of |D D D| in the same normalisation (the rounding-error scale
    of any summation order), and the per-triangle relative errors."""
    b = np.asarray(b, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = np.abs(b - ref)
    out = dict(e_norm=float(np.linalg.norm(b - ref) / np.linalg.norm(ref)),
               e_strict_max=float(np.max(d / np.abs(ref))),
               e_strict_med=float(np.median(d / np.abs(ref))))
    if s_abs is not None:
        out["e_cond"] = float(np.max(d / np.asarray(s_abs)))
    return out
