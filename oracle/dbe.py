"""Direct bispectrum estimator: the closed-triangle triple sum written out.

TEST INFRASTRUCTURE ONLY (see the package docstring).

This is the definition the fast estimator must reproduce exactly (eq. binbs and
eq. Ntri1 of Section 2.1): for a bin (a1, a2, a3),
    B = (V N_tri)^-1 sum_{k1 in a1} sum_{k2 in a2} sum_{k3 in a3}
            Delta(k1) Delta(k2) Delta(k3) delta_K(k1 + k2 + k3),
    N_tri = the number of ordered (k1, k2, k3) with k1 + k2 + k3 = 0.
As in the paper's description of the direct method, it loops over the modes
of shells a2 and a3 and keeps the pairs whose closing mode -(k2 + k3) lies in
shell a1.  No wrap-around: the closing mode is the true lattice vector.  Cost
is N_a2 N_a3 per bin, so it is meant for grids of 24^3 or smaller.
"""
from __future__ import annotations

import numpy as np

from . import geometry


def full_spectrum(delta: np.ndarray, box_l: float, rsd_beta: float = 0.0) -> np.ndarray:
    """Delta(k) = dV * fftn(delta) on the full grid, times (1 + beta mu_k^2)."""
    n_g = delta.shape[0]
    dv = (box_l / n_g) ** 3
    spec = np.fft.fftn(np.asarray(delta, dtype=np.float64)) * dv
    if rsd_beta != 0.0:
        m = np.fft.fftfreq(n_g, d=1.0 / n_g)
        mx, my, mz = np.meshgrid(m, m, m, indexing="ij")
        m2 = mx * mx + my * my + mz * mz
        mu2 = np.where(m2 > 0, mz * mz / np.where(m2 > 0, m2, 1.0), 0.0)
        spec = spec * (1.0 + rsd_beta * mu2)
    return spec


def shell_modes(w: float, n_shells: int):
    """{n: integer mode vectors (M, 3) of shell n} over the whole lattice."""
    pts = geometry.lattice_ball((n_shells + 0.5) * w + 1.0)
    s = geometry.shell_of_m2((pts * pts).sum(1), w, n_shells)
    return {n: pts[s == n] for n in range(1, n_shells + 1)}


def _lookup(spec: np.ndarray, m: np.ndarray) -> np.ndarray:
    n_g = spec.shape[0]
    idx = np.mod(m, n_g)
    return spec[idx[..., 0], idx[..., 1], idx[..., 2]]


def estimate(delta: np.ndarray, box_l: float, w: float, triangles: np.ndarray,
             rsd_beta: float = 0.0) -> dict:
    """Brute-force B (real part), the imaginary part, and N_tri per triangle."""
    delta = np.asarray(delta, dtype=np.float64)
    n_g = delta.shape[0]
    tri = np.asarray(triangles, dtype=np.int64).reshape(-1, 3)
    n_s = int(tri.max())
    spec = full_spectrum(delta, box_l, rsd_beta)
    modes = shell_modes(w, n_s)
    vol = box_l ** 3
    B = np.zeros(len(tri))
    B_imag = np.zeros(len(tri))
    ntri = np.zeros(len(tri), dtype=np.int64)
    for t, (a1, a2, a3) in enumerate(tri):
        m2v, m3v = modes[int(a2)], modes[int(a3)]
        k1 = -(m2v[:, None, :] + m3v[None, :, :])            # closing mode
        in_a1 = geometry.shell_of_m2((k1 * k1).sum(-1), w, n_s) == a1
        i2, i3 = np.nonzero(in_a1)
        if len(i2) and np.any(np.abs(k1[i2, i3]) >= n_g // 2):
            raise ValueError("closing mode outside the grid's unique range")
        prod = (_lookup(spec, k1[i2, i3]) * _lookup(spec, m2v[i2]) * _lookup(spec, m3v[i3]))
        total = prod.sum()
        ntri[t] = len(i2)
        if ntri[t]:
            B[t] = total.real / (vol * ntri[t])
            B_imag[t] = total.imag / (vol * ntri[t])
        else:
            B[t] = B_imag[t] = np.nan
    return dict(B=B, B_imag=B_imag, ntri=ntri)


def gradient(delta: np.ndarray, box_l: float, w: float, triangles: np.ndarray,
             weights: np.ndarray, rsd_beta: float = 0.0) -> np.ndarray:
    """d(sum_t v_t B_t)/d delta(x) from the direct sum: with
    dDelta(k)/d delta(x) = dV e^{-ik.x}, each closed triangle contributes
    dV Re[Z1 e^{-ik1.x} Delta2 Delta3 + Delta1 Z2 e^{-ik2.x} Delta3
    + Delta1 Delta2 Z3 e^{-ik3.x}] / (V N_tri), where Delta already holds the
    RSD factors Z and the e^{-ik.x} terms carry their own Z."""
    delta = np.asarray(delta, dtype=np.float64)
    n_g = delta.shape[0]
    dv = (box_l / n_g) ** 3
    vol = box_l ** 3
    tri = np.asarray(triangles, dtype=np.int64).reshape(-1, 3)
    n_s = int(tri.max())
    spec = full_spectrum(delta, box_l, rsd_beta)
    m = np.fft.fftfreq(n_g, d=1.0 / n_g)
    mx, my, mz = np.meshgrid(m, m, m, indexing="ij")
    m2 = mx * mx + my * my + mz * mz
    zfac = 1.0 + rsd_beta * np.where(m2 > 0, mz * mz / np.where(m2 > 0, m2, 1.0), 0.0)
    modes = shell_modes(w, n_s)
    # accumulate c(k) = sum over triangles of the coefficient multiplying e^{-ik.x}
    coef = np.zeros((n_g, n_g, n_g), dtype=np.complex128)
    for t, (a1, a2, a3) in enumerate(tri):
        m2v, m3v = modes[int(a2)], modes[int(a3)]
        k1 = -(m2v[:, None, :] + m3v[None, :, :])
        i2, i3 = np.nonzero(geometry.shell_of_m2((k1 * k1).sum(-1), w, n_s) == a1)
        n_t = len(i2)
        if n_t == 0:
            continue
        c = weights[t] / (vol * n_t)
        v1, v2, v3 = k1[i2, i3], m2v[i2], m3v[i3]
        d1, d2, d3 = _lookup(spec, v1), _lookup(spec, v2), _lookup(spec, v3)
        for vec, other in ((v1, d2 * d3), (v2, d1 * d3), (v3, d1 * d2)):
            idx = np.mod(vec, n_g)
            np.add.at(coef, (idx[:, 0], idx[:, 1], idx[:, 2]),
                      c * other * zfac[idx[:, 0], idx[:, 1], idx[:, 2]])
    # sum_k coef(k) e^{-ik.x} = fftn(coef) evaluated at x
    return dv * np.real(np.fft.fftn(coef))
