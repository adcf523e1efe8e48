"""Analytic predictions used to pin the oracle statistically.

TEST INFRASTRUCTURE ONLY (see the package docstring).

  * Tree-level bispectrum of the quadratic non-Gaussian field (eq. bana):
        B = 2 f_NG [P(k1)P(k2) + P(k2)P(k3) + P(k3)P(k1)],
    exact at linear order in f_NG on the periodic grid as well.
  * Its exact bin average (eq. binavgbs): the mean of B over the closed
    triangles of the bin, computed with P-weighted unit fields
        I^w_n(x) = sum_{k in n} w(k) e^{ik.x}
    so that sum_{closed} P1 P2 = N^-3 sum_x I^P_a1 I^P_a2 I_a3, etc.
  * Linear RSD (eq. RSD) multiplies each Delta by Z(k) = 1 + beta mu_k^2 with
    mu_k = k_z/|k|.  The monopole of the redshift-space bispectrum is the
    orientation average of Z1 Z2 Z3 times B.  Averaging products of (z.u)^2
    over isotropic directions (the 2nd, 4th and 6th moments of a unit
    vector: 1/3, (1 + 2 c^2)/15 and (1 + 2 S + 8 c12 c23 c31)/105) gives
        R(beta) = 1 + beta + beta^2 (3 + 2 S)/15
                  + beta^3 (1 + 2 S + 8 c12 c23 c31)/105,
    with c_ab = khat_a . khat_b of the closed triangle and
    S = c12^2 + c23^2 + c31^2.  Bin-averaged, Z enters the weighted unit fields.
"""
from __future__ import annotations

import numpy as np

from . import fbe


def b_tree(k1, k2, k3, power, f_ng: float):
    p1, p2, p3 = power(k1), power(k2), power(k3)
    return 2.0 * f_ng * (p1 * p2 + p2 * p3 + p3 * p1)


def _weighted_unit_field(weight_half: np.ndarray, mask: np.ndarray) -> np.ndarray:
    n_g = mask.shape[0]
    return fbe._irfftn(np.where(mask, weight_half, 0.0).astype(np.complex128),
                       s=(n_g, n_g, n_g)) * float(n_g) ** 3


def b_tree_binavg(n_g: int, box_l: float, w: float, triangles, power, f_ng: float,
                  rsd_beta: float = 0.0) -> np.ndarray:
    """Exact mean of Z1 Z2 Z3 B_tree over the closed triangles of each bin."""
    tri = np.asarray(triangles, dtype=np.int64).reshape(-1, 3)
    shells = sorted(set(int(v) for v in tri.ravel()))
    masks = fbe.shell_masks(n_g, w, shells)
    kf = 2.0 * np.pi / box_l
    kmag = kf * np.sqrt(fbe.half_grid_m2(n_g).astype(np.float64))
    pk = power(kmag)
    z = fbe.rsd_factor(n_g, rsd_beta) if rsd_beta != 0.0 else np.ones_like(kmag)
    IP = {n: _weighted_unit_field(z * pk, masks[n]) for n in shells}
    IZ = {n: _weighted_unit_field(z, masks[n]) for n in shells}
    I1 = {n: fbe.unit_field(masks[n]) for n in shells}
    out = np.zeros(len(tri))
    for t, (a1, a2, a3) in enumerate(tri):
        a1, a2, a3 = int(a1), int(a2), int(a3)
        s = (np.sum(IP[a1] * IP[a2] * IZ[a3]) + np.sum(IZ[a1] * IP[a2] * IP[a3])
             + np.sum(IP[a1] * IZ[a2] * IP[a3]))
        ntri = np.rint(np.sum(I1[a1] * I1[a2] * I1[a3]) / float(n_g) ** 3)
        out[t] = 2.0 * f_ng * s / (float(n_g) ** 3 * ntri)
    return out


def triangle_cosines(k1, k2, k3):
    """c12, c23, c31 = khat_a . khat_b for a closed triangle k1 + k2 + k3 = 0."""
    c12 = (k3 * k3 - k1 * k1 - k2 * k2) / (2.0 * k1 * k2)
    c23 = (k1 * k1 - k2 * k2 - k3 * k3) / (2.0 * k2 * k3)
    c31 = (k2 * k2 - k3 * k3 - k1 * k1) / (2.0 * k3 * k1)
    return c12, c23, c31


def rsd_monopole_factor(k1, k2, k3, beta: float):
    """R(beta) above for side lengths (k1, k2, k3)."""
    c12, c23, c31 = triangle_cosines(k1, k2, k3)
    S = c12 * c12 + c23 * c23 + c31 * c31
    return (1.0 + beta + beta * beta * (3.0 + 2.0 * S) / 15.0
            + beta ** 3 * (1.0 + 2.0 * S + 8.0 * c12 * c23 * c31) / 105.0)


def rsd_monopole_factor_mc(k1, k2, k3, beta: float, n_dirs: int, seed: int = 0):
    """The same orientation average by Monte Carlo over random rotations
    (an independent check of the closed form)."""
    rng = np.random.default_rng(seed)
    c12 = (k3 * k3 - k1 * k1 - k2 * k2) / (2.0 * k1 * k2)
    s12 = np.sqrt(max(0.0, 1.0 - c12 * c12))
    v1 = np.array([k1, 0.0, 0.0])
    v2 = k2 * np.array([c12, s12, 0.0])
    v3 = -(v1 + v2)
    q = rng.standard_normal((n_dirs, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    a, b, c, d = q.T
    # third row of the rotation matrix of each unit quaternion = image of z
    zrow = np.stack([2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d], 1)
    prod = np.ones(n_dirs)
    for v in (v1, v2, v3):
        mu = zrow @ v / np.linalg.norm(v)
        prod *= 1.0 + beta * mu * mu
    return float(prod.mean()), float(prod.std() / np.sqrt(n_dirs))


def gaussian_variance_binavg(n_g: int, box_l: float, w: float, triangles, power) -> np.ndarray:
    """Variance of the estimated B of a Gaussian field (B = 0) in bins of three
    distinct shells: the Gaussian term of eq. cv, V P1 P2 P3 / N_tri, with the
    product averaged over the closed triangles of the bin (only the pairing of
    each triangle with its mirror image survives when the shells differ):
        Var B = V N^-3 sum_x I^P_a1 I^P_a2 I^P_a3 / N_tri^2,
    I^P the P-weighted unit fields.  Bins with repeated shells have extra
    pairings (eq. cv carries no symmetry factor) and are rejected."""
    tri = np.asarray(triangles, dtype=np.int64).reshape(-1, 3)
    if np.any((tri[:, 0] == tri[:, 1]) | (tri[:, 1] == tri[:, 2])):
        raise ValueError("bins with repeated shells have extra pairings")
    shells = sorted(set(int(v) for v in tri.ravel()))
    masks = fbe.shell_masks(n_g, w, shells)
    kf = 2.0 * np.pi / box_l
    pk = power(kf * np.sqrt(fbe.half_grid_m2(n_g).astype(np.float64)))
    IP = {n: _weighted_unit_field(pk, masks[n]) for n in shells}
    I1 = {n: fbe.unit_field(masks[n]) for n in shells}
    vol = box_l ** 3
    out = np.zeros(len(tri))
    for t, (a1, a2, a3) in enumerate(tri):
        a1, a2, a3 = int(a1), int(a2), int(a3)
        ntri = np.rint(np.sum(I1[a1] * I1[a2] * I1[a3]) / float(n_g) ** 3)
        out[t] = vol * np.sum(IP[a1] * IP[a2] * IP[a3]) / float(n_g) ** 3 / ntri ** 2
    return out
