"""Gradient of a weighted sum of the FBE output with respect to delta(x).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For L = sum_t v_t B_t with B_t = T_t / (V N_tri,t N^3) and
T_t = sum_x D_a1 D_a2 D_a3 (eq. bsfin), D_n(x) = sum_{k in n} Z(k) Delta(k) e^{ik.x}
(eq. iFT with the RSD factor Z of eq. RSD), Delta(k) = dV sum_y delta(y) e^{-ik.y}:
  c_t   = v_t / (V N_tri,t N^3)
  G_n(x) = sum_t c_t ([n = a1] D_a2 D_a3 + [n = a2] D_a1 D_a3 + [n = a3] D_a1 D_a2)
  dL/d delta(y) = dV sum_n sum_{k in n} Z(k) G^_n(k) e^{ik.y},  G^_n = DFT(G_n)
               = dV N^3 irfftn( sum_n mask_n Z rfftn(G_n) ).
(The chain rule through the real field D_n; the shells are symmetric under
k -> -k and Z is even, which turns the adjoint's e^{-ik.y} into e^{+ik.y}.)
"""
from __future__ import annotations

import numpy as np

from . import fbe


def gradient(delta: np.ndarray, box_l: float, w: float, triangles: np.ndarray,
             weights: np.ndarray, rsd_beta: float = 0.0, ntri=None) -> np.ndarray:
    delta = np.asarray(delta, dtype=np.float64)
    n_g = delta.shape[0]
    tri = np.asarray(triangles, dtype=np.int64).reshape(-1, 3)
    if ntri is None:
        ntri = fbe.estimate(delta, box_l, w, tri, rsd_beta)["ntri"]
    vol = box_l ** 3
    dv = vol / n_g ** 3
    shells = sorted(set(int(v) for v in tri.ravel()))
    masks = fbe.shell_masks(n_g, w, shells)
    spec = fbe.spectrum(delta, box_l, rsd_beta)
    D = {n: fbe.shell_field(spec, masks[n]) for n in shells}
    c = np.asarray(weights, dtype=np.float64) / (vol * ntri.astype(np.float64) * float(n_g) ** 3)
    G = {n: np.zeros_like(D[n]) for n in shells}
    for ct, (a1, a2, a3) in zip(c, tri):
        a1, a2, a3 = int(a1), int(a2), int(a3)
        G[a1] += ct * D[a2] * D[a3]
        G[a2] += ct * D[a1] * D[a3]
        G[a3] += ct * D[a1] * D[a2]
    zfac = fbe.rsd_factor(n_g, rsd_beta) if rsd_beta != 0.0 else 1.0
    acc = np.zeros(spec.shape, dtype=np.complex128)
    for n in shells:
        acc += np.where(masks[n], fbe._rfftn(G[n]), 0.0)
    acc *= zfac
    return dv * float(n_g) ** 3 * fbe._irfftn(acc, s=(n_g, n_g, n_g))
