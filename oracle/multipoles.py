"""Multipoles of the redshift-space bispectrum in float64 (line of sight z).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 3.1 applies the method to the redshift-space field (eq. RSD, line of
sight z) and estimates the monopole.  Its higher moments in the orientation of
the triangle are the Legendre moments in the angle between the first side and
the line of sight (reading: the weight sits on the first shell a1 of the bin,
mu_1 = k1_z / |k1|, and l is even):

    B_l(a1, a2, a3) = (2 l + 1) (V N_tri)^-1
        sum_{k1 in a1, k2 in a2, k3 in a3, k1 + k2 + k3 = 0} L_l(mu_1) Delta(k1) Delta(k2) Delta(k3),

so that l = 0 is eq. bsfin.  In grid-sum form the weight goes into the a1
shell field, D^l_n(x) = sum_{k in n} L_l(mu_k) Delta(k) e^{i k.x} (eq. iFT with
a weight), and

    B_l = (2 l + 1) sum_x D^l_a1(x) D_a2(x) D_a3(x) / (V N_tri N^3),

with N_tri the unweighted count (eqs. Ntri1, Ntri2).  For odd l the weighted
closed sum of a real field is purely imaginary (k -> -k flips L_l), so only
l = 0, 2, 4 are defined here.

  legendre          L_l(mu) for l = 0, 2, 4
  estimate          the grid-sum form (numpy FFTs, float64)
  direct_estimate   the weighted closed-triangle sum written out (small grids)
"""
from __future__ import annotations

import numpy as np

from . import dbe, fbe, geometry

ELLS = (0, 2, 4)


def legendre(ell: int, mu: np.ndarray) -> np.ndarray:
    """Legendre polynomial L_l(mu), l in {0, 2, 4}."""
    mu = np.asarray(mu, dtype=np.float64)
    if ell == 0:
        return np.ones_like(mu)
    if ell == 2:
        return 0.5 * (3.0 * mu * mu - 1.0)
    if ell == 4:
        mu2 = mu * mu
        return (35.0 * mu2 * mu2 - 30.0 * mu2 + 3.0) / 8.0
    raise ValueError("multipole order must be 0, 2 or 4")


def _mu_half(n_g: int) -> np.ndarray:
    """mu = m_z / |m| on the rfftn half spectrum (0 at m = 0)."""
    mx, my, mz = fbe.half_grid_m(n_g)
    m2 = (mx * mx + my * my + mz * mz).astype(np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(m2 > 0, mz / np.sqrt(np.where(m2 > 0, m2, 1.0)), 0.0)


def estimate(delta: np.ndarray, box_l: float, w: float, triangles: np.ndarray, ell: int,
             rsd_beta: float = 0.0, with_abs: bool = False, ntri_tol: float = 1e-3) -> dict:
    """B_l per bin (grid sums on the full grid), N_tri, and optionally the
    summation scale S = (2 l + 1) sum_x |D^l D D| / (V N_tri N^3)."""
    if ell not in ELLS:
        raise ValueError("multipole order must be 0, 2 or 4")
    delta = np.asarray(delta, dtype=np.float64)
    n_g = delta.shape[0]
    tri = np.asarray(triangles, dtype=np.int64).reshape(-1, 3)
    n_s = int(tri.max())
    if not geometry.check_cutoff(n_g, w, n_s):
        raise ValueError("shell modes reach beyond 2 pi N_g / (3 L)")
    shells = sorted(set(int(v) for v in tri.ravel()))
    firsts = sorted(set(int(v) for v in tri[:, 0]))
    masks = fbe.shell_masks(n_g, w, shells)
    spec = fbe.spectrum(delta, box_l, rsd_beta)
    wspec = spec * legendre(ell, _mu_half(n_g))
    # weighted first-side fields under keys -n, the plain fields under n
    keys = [-n for n in firsts] + shells
    stack = np.empty((len(keys), n_g ** 3), dtype=np.float64)
    for r, key in enumerate(keys):
        src = wspec if key < 0 else spec
        stack[r] = fbe.shell_field(src, masks[abs(key)]).ravel()
    pos = {key: r for r, key in enumerate(keys)}
    wtri = tri.copy()
    wtri[:, 0] = -wtri[:, 0]
    T = fbe.triple_sums((stack, pos), wtri)
    S = fbe.abs_triple_sums((stack, pos), wtri) if with_abs else None
    del stack
    ufields = fbe._field_stack(lambda n: fbe.unit_field(masks[n]), shells, n_g ** 3)
    raw = fbe.triple_sums(ufields, tri) / float(n_g) ** 3
    del ufields
    ntri = np.rint(raw).astype(np.int64)
    if len(raw) and float(np.max(np.abs(raw - ntri))) > ntri_tol:
        raise AssertionError("N_tri sums are not integers")
    vol = box_l ** 3
    with np.errstate(invalid="ignore", divide="ignore"):
        norm = (2.0 * ell + 1.0) / (vol * ntri.astype(np.float64) * float(n_g) ** 3)
        out = dict(B=T * norm, ntri=ntri)
        if with_abs:
            out["S"] = S * norm
    return out


def direct_estimate(delta: np.ndarray, box_l: float, w: float, triangles: np.ndarray, ell: int,
                    rsd_beta: float = 0.0) -> dict:
    """The weighted closed-triangle sum: for every k2 in a2 and k3 in a3, the
    closing k1 = -(k2 + k3) as a true lattice vector, kept when it lies in a1,
    weighted by L_l(k1_z / |k1|).  Returns B_l (real part), its imaginary part
    and N_tri."""
    delta = np.asarray(delta, dtype=np.float64)
    n_g = delta.shape[0]
    tri = np.asarray(triangles, dtype=np.int64).reshape(-1, 3)
    n_s = int(tri.max())
    spec = dbe.full_spectrum(delta, box_l, rsd_beta)
    modes = dbe.shell_modes(w, n_s)
    vol = box_l ** 3

    def at(m):
        idx = np.mod(m, n_g)
        return spec[idx[..., 0], idx[..., 1], idx[..., 2]]

    B = np.full(len(tri), np.nan)
    B_imag = np.full(len(tri), np.nan)
    ntri = np.zeros(len(tri), dtype=np.int64)
    for t, (a1, a2, a3) in enumerate(tri):
        k2, k3 = modes[int(a2)], modes[int(a3)]
        k1 = -(k2[:, None, :] + k3[None, :, :])
        keep = geometry.shell_of_m2((k1 * k1).sum(-1), w, n_s) == a1
        i2, i3 = np.nonzero(keep)
        k1 = k1[i2, i3]
        if len(k1) and np.any(np.abs(k1) >= n_g // 2):
            raise ValueError("closing mode outside the grid's unique range")
        mu1 = k1[:, 2] / np.sqrt((k1 * k1).sum(-1).astype(np.float64))
        total = (legendre(ell, mu1) * at(k1) * at(k2[i2]) * at(k3[i3])).sum()
        ntri[t] = len(k1)
        if ntri[t]:
            B[t] = (2 * ell + 1) * total.real / (vol * ntri[t])
            B_imag[t] = (2 * ell + 1) * total.imag / (vol * ntri[t])
    return dict(B=B, B_imag=B_imag, ntri=ntri)
