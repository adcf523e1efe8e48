"""The FFT-based bispectrum estimator in float64 (numpy / scipy.fft).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Section 2.2 of the paper step by step:
  1. Delta(k) = dV * sum_x delta(x) exp(-i k.x)          (the Fourier convention
     fixed by eq. bs: <Delta Delta Delta> = V B), times the linear-RSD factor
     (1 + beta mu_k^2) with the line of sight along z (eq. RSD) when beta != 0;
  2. per shell n, the real field D_n(x) = sum_{k in n} Delta(k) exp(+i k.x)
     (eq. iFT; the shells are symmetric under k -> -k and Delta(-k) = Delta*(k),
     so the sign of the exponent does not change D_n), computed as
     N^3 * irfftn(mask_n * Delta);
  3. per shell n, the unit field I_n(x) = sum_{k in n} exp(+i k.x) (eq. 2FT);
  4. T = sum_x D_a1 D_a2 D_a3 per triangle (numerator of eq. bsfin), with one
     library matmul per shell pair (a1, a2) over the a3 of that pair;
  5. N_tri = N^-3 sum_x I_a1 I_a2 I_a3 (eq. Ntri2), rounded to the integer it
     must be, with the residue reported;
  6. B = T / (V N_tri N^3) (eq. bsfin).
"""
from __future__ import annotations

import math

import numpy as np

from . import geometry

try:
    import scipy.fft as _sfft

    def _rfftn(a):
        return _sfft.rfftn(a, workers=-1)

    def _irfftn(a, s):
        return _sfft.irfftn(a, s=s, workers=-1)
except Exception:  # pragma: no cover
    def _rfftn(a):
        return np.fft.rfftn(a)

    def _irfftn(a, s):
        return np.fft.irfftn(a, s=s)


def half_grid_m(n_g: int):
    """Integer (mx, my, mz) broadcastable over the rfftn half spectrum [N][N][N/2+1]."""
    m = np.fft.fftfreq(n_g, d=1.0 / n_g).astype(np.int64)
    mz = np.arange(n_g // 2 + 1, dtype=np.int64)
    return m[:, None, None], m[None, :, None], mz[None, None, :]


def half_grid_m2(n_g: int) -> np.ndarray:
    mx, my, mz = half_grid_m(n_g)
    return mx * mx + my * my + mz * mz


def rsd_factor(n_g: int, beta: float) -> np.ndarray:
    """1 + beta (k_z/|k|)^2 on the half spectrum (line of sight = z); 1 at k = 0."""
    mx, my, mz = half_grid_m(n_g)
    m2 = (mx * mx + my * my + mz * mz).astype(np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        mu2 = np.where(m2 > 0, (mz * mz) / np.where(m2 > 0, m2, 1.0), 0.0)
    return 1.0 + beta * mu2


def spectrum(delta: np.ndarray, box_l: float, rsd_beta: float = 0.0) -> np.ndarray:
    """Delta(k) on the half spectrum: dV * rfftn(delta), times the RSD factor."""
    n_g = delta.shape[0]
    dv = (box_l / n_g) ** 3
    spec = _rfftn(np.asarray(delta, dtype=np.float64)) * dv
    if rsd_beta != 0.0:
        spec *= rsd_factor(n_g, rsd_beta)
    return spec


def shell_masks(n_g: int, w: float, shells):
    s = geometry.shell_of_m2(half_grid_m2(n_g), w, max(shells))
    return {n: (s == n) for n in shells}


def shell_field(spec: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """D_n(x) = sum_{k in shell} Delta(k) e^{ik.x} = N^3 irfftn(mask * Delta)."""
    n_g = spec.shape[0]
    return _irfftn(np.where(mask, spec, 0.0), s=(n_g, n_g, n_g)) * float(n_g) ** 3


def shell_field_at(spec: np.ndarray, mask: np.ndarray, n_eval: int) -> np.ndarray:
    """D_n at the points x_j = L j / n_eval (j in [0, n_eval)^3) of a grid other
    than the input one: the same mode sum, sum_{k in shell} Delta(k) e^{ik.x_j},
    evaluated by placing each shell mode at its signed frequency in an n_eval
    half spectrum (every mode must satisfy |m_i| < n_eval / 2)."""
    n_g = spec.shape[0]
    mx, my, mz = half_grid_m(n_g)
    sel = np.nonzero(mask)
    fx, fy, fz = mx.ravel()[sel[0]], my.ravel()[sel[1]], mz.ravel()[sel[2]]
    if len(fx) and max(np.abs(fx).max(), np.abs(fy).max(), fz.max()) * 2 >= n_eval:
        raise ValueError("shell modes do not fit the evaluation grid")
    out = np.zeros((n_eval, n_eval, n_eval // 2 + 1), dtype=np.complex128)
    out[fx % n_eval, fy % n_eval, fz] = spec[sel]
    return _irfftn(out, s=(n_eval,) * 3) * float(n_eval) ** 3


def unit_field(mask: np.ndarray) -> np.ndarray:
    """I_n(x) = sum_{k in shell} e^{ik.x} = N^3 irfftn(mask)."""
    n_g = mask.shape[0]
    return _irfftn(mask.astype(np.complex128), s=(n_g, n_g, n_g)) * float(n_g) ** 3


def _as_stack(fields):
    """(stack, pos): the fields as rows of one 2-D array and shell -> row."""
    if isinstance(fields, tuple):
        return fields
    keys = sorted(fields)
    stack = np.stack([np.asarray(fields[k], dtype=np.float64).ravel() for k in keys])
    return stack, {k: r for r, k in enumerate(keys)}


def triple_sums(fields, triangles: np.ndarray) -> np.ndarray:
    """sum_x f_a1 f_a2 f_a3 for every row (a1, a2, a3); one product field per
    distinct (a1, a2) and one matmul over that pair's a3 values.  `fields` is
    a dict shell -> field or a (stack, pos) pair of a 2-D array whose rows are
    the fields and the shell -> row map (a pair's a3 rows are then read as a
    view when they are consecutive rows, without a copy)."""
    stack, pos = _as_stack(fields)
    tri = np.asarray(triangles)
    out = np.zeros(len(tri), dtype=np.float64)
    pairs = {}
    for idx, (a1, a2, a3) in enumerate(tri):
        pairs.setdefault((int(a1), int(a2)), []).append((pos[int(a3)], idx))
    prod = np.empty(stack.shape[1], dtype=np.float64)
    for (a1, a2), rows in pairs.items():
        np.multiply(stack[pos[a1]], stack[pos[a2]], out=prod)
        rows.sort()
        r = [q for q, _ in rows]
        if r[-1] - r[0] == len(r) - 1:
            out[[i for _, i in rows]] = stack[r[0]:r[-1] + 1] @ prod
        else:
            for q, i in rows:
                out[i] = stack[q] @ prod
    return out


def abs_triple_sums(fields, triangles: np.ndarray) -> np.ndarray:
    """sum_x |f_a1 f_a2 f_a3| (the summation-condition denominator)."""
    stack, pos = _as_stack(fields)
    return triple_sums((np.abs(stack), pos), triangles)


def _field_stack(make, shells, n_vox):
    """(stack, pos) with row r = make(shells[r]) flattened."""
    stack = np.empty((len(shells), n_vox), dtype=np.float64)
    for r, n in enumerate(shells):
        stack[r] = make(n).ravel()
    return stack, {n: r for r, n in enumerate(shells)}


def estimate(delta: np.ndarray, box_l: float, w: float, triangles: np.ndarray,
             rsd_beta: float = 0.0, enforce_cutoff: bool = True,
             with_abs: bool = False, ntri_tol: float = 1e-3) -> dict:
    """Full FBE in float64.  Returns B, ntri (int64), T, the raw N_tri sums,
    and (optionally) S = sum|D D D| / (V N_tri N^3)."""
    delta = np.asarray(delta, dtype=np.float64)
    n_g = delta.shape[0]
    tri = np.asarray(triangles, dtype=np.int64).reshape(-1, 3)
    n_s = int(tri.max()) if len(tri) else 1
    if enforce_cutoff and not geometry.check_cutoff(n_g, w, n_s):
        raise ValueError("shell modes reach beyond 2 pi N_g / (3 L)")
    shells = sorted(set(int(v) for v in tri.ravel()))
    masks = shell_masks(n_g, w, shells)
    spec = spectrum(delta, box_l, rsd_beta)
    dfields = _field_stack(lambda n: shell_field(spec, masks[n]), shells, n_g ** 3)
    T = triple_sums(dfields, tri)
    S = abs_triple_sums(dfields, tri) if with_abs else None
    del dfields
    ufields = _field_stack(lambda n: unit_field(masks[n]), shells, n_g ** 3)
    raw = triple_sums(ufields, tri) / float(n_g) ** 3
    del ufields
    ntri = np.rint(raw).astype(np.int64)
    resid = float(np.max(np.abs(raw - ntri))) if len(raw) else 0.0
    if resid > ntri_tol:
        raise AssertionError("N_tri sums are not integers: residue %g" % resid)
    vol = box_l ** 3
    with np.errstate(invalid="ignore", divide="ignore"):
        norm = 1.0 / (vol * ntri.astype(np.float64) * float(n_g) ** 3)
        B = T * norm
        out = dict(B=B, ntri=ntri, T=T, ntri_raw=raw, ntri_resid=resid)
        if with_abs:
            out["S"] = S * norm
    return out
