"""The fourth-order polyspectrum (trispectrum) estimator in float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 4 of the paper extends the method to the p-th order polyspectrum and
states its aliasing cutoff, k < 2 pi N_g / (p L): the grid sum of p shell
fields picks mode p-tuples with k_1 + ... + k_p = 0 modulo the grid, which is
exactly the closed ones while p max|m_i| < N_g.  For p = 4 the estimator of a
bin of four shells (a1 >= a2 >= a3 >= a4) is the bispectrum's written with four
fields (reading: the same normalisation as eq. bsfin, one more factor):

    T = (V N_quad)^-1 sum_{closed (k1, k2, k3, k4)} Delta_1 Delta_2 Delta_3 Delta_4
      = (V N_quad N_g^3)^-1 sum_x D_a1(x) D_a2(x) D_a3(x) D_a4(x),
    N_quad = the number of ordered closed 4-tuples = N_g^-3 sum_x I_a1 I_a2 I_a3 I_a4,

with D_n and I_n the shell and unit fields of eqs. iFT and 2FT.  It is the
bin average of the full four-point function (the paper defines no subtraction
of its Gaussian part).  A bin can close when a2 + a3 + a4 >= a1 (the
largest side no longer than the sum of the others, as eq. cond for three).

  fft_estimate      the grid-sum form above (numpy FFTs, float64);
  direct_estimate   the closed-4-tuple sum written out (grids of 16^3 or smaller).
"""
from __future__ import annotations

import numpy as np

from . import dbe, fbe, geometry


def all_quads(n_shells: int, k1_set=None) -> np.ndarray:
    """All closable shell quadruples a1 >= a2 >= a3 >= a4 >= 1 with
    a2 + a3 + a4 >= a1, ascending; optionally only a1 in k1_set.  int32 (Q, 4)."""
    keep = None if k1_set is None else set(int(a) for a in k1_set)
    rows = []
    for a1 in range(1, n_shells + 1):
        if keep is not None and a1 not in keep:
            continue
        for a2 in range(1, a1 + 1):
            for a3 in range(1, a2 + 1):
                for a4 in range(1, a3 + 1):
                    if a2 + a3 + a4 >= a1:
                        rows.append((a1, a2, a3, a4))
    return np.array(rows, dtype=np.int32).reshape(-1, 4)


def check_cutoff(n_g: int, w: float, n_shells: int, p: int = 4) -> bool:
    """True when every shell mode lies below 2 pi N_g/(p L): (n_s + 1/2) w p <= N_g."""
    return (n_shells + 0.5) * w * p <= n_g


def fft_estimate(delta: np.ndarray, box_l: float, w: float, quads: np.ndarray, rsd_beta: float = 0.0,
                 enforce_cutoff: bool = True, with_abs: bool = False, ntri_tol: float = 1e-3) -> dict:
    """T (four-field grid sum), N_quad (rounded, with its residue) and, if asked,
    S = sum_x |D D D D| in the same normalisation."""
    delta = np.asarray(delta, dtype=np.float64)
    n_g = delta.shape[0]
    q = np.asarray(quads, dtype=np.int64).reshape(-1, 4)
    n_s = int(q.max()) if len(q) else 1
    if enforce_cutoff and not check_cutoff(n_g, w, n_s):
        raise ValueError("shell modes reach beyond 2 pi N_g / (4 L)")
    shells = sorted(set(int(v) for v in q.ravel()))
    masks = fbe.shell_masks(n_g, w, shells)
    spec = fbe.spectrum(delta, box_l, rsd_beta)

    def sums(field_of):
        f = {n: field_of(n) for n in shells}
        out = np.zeros(len(q))
        pair = {}
        for t, (a1, a2, a3, a4) in enumerate(q):
            k12, k34 = (int(a1), int(a2)), (int(a3), int(a4))
            for k in (k12, k34):
                if k not in pair:
                    pair[k] = (f[k[0]] * f[k[1]]).ravel()
            out[t] = pair[k12] @ pair[k34]
        return out

    D = {n: fbe.shell_field(spec, masks[n]) for n in shells}
    T = sums(lambda n: D[n])
    S = sums(lambda n: np.abs(D[n])) if with_abs else None
    del D
    raw = sums(lambda n: fbe.unit_field(masks[n])) / float(n_g) ** 3
    nq = np.rint(raw).astype(np.int64)
    resid = float(np.max(np.abs(raw - nq))) if len(raw) else 0.0
    if resid > ntri_tol:
        raise AssertionError("N_quad sums are not integers: residue %g" % resid)
    vol = box_l ** 3
    with np.errstate(invalid="ignore", divide="ignore"):
        norm = 1.0 / (vol * nq.astype(np.float64) * float(n_g) ** 3)
        out = dict(T4=T * norm, nquad=nq, raw=raw, resid=resid)
        if with_abs:
            out["S"] = S * norm
    return out


def direct_estimate(delta: np.ndarray, box_l: float, w: float, quads: np.ndarray, rsd_beta: float = 0.0) -> dict:
    """The closed-4-tuple sum: for every k1 in a1, k2 in a2, k3 in a3, the
    closing k4 = -(k1 + k2 + k3) as a true lattice vector (no wrap-around),
    kept when it lies in a4.  Returns T4 (real part), its imaginary part and
    N_quad."""
    delta = np.asarray(delta, dtype=np.float64)
    q = np.asarray(quads, dtype=np.int64).reshape(-1, 4)
    n_s = int(q.max())
    spec = dbe.full_spectrum(delta, box_l, rsd_beta)
    modes = dbe.shell_modes(w, n_s)
    vol = box_l ** 3
    T = np.zeros(len(q))
    T_im = np.zeros(len(q))
    nq = np.zeros(len(q), dtype=np.int64)
    n_g = delta.shape[0]

    def val(m):
        i = np.mod(m, n_g)
        return spec[i[..., 0], i[..., 1], i[..., 2]]

    for t, (a1, a2, a3, a4) in enumerate(q):
        m1, m2, m3 = modes[int(a1)], modes[int(a2)], modes[int(a3)]
        v1, v2, v3 = val(m1), val(m2), val(m3)
        acc = 0.0 + 0.0j
        cnt = 0
        s23 = m2[:, None, :] + m3[None, :, :]                 # (M2, M3, 3)
        v23 = v2[:, None] * v3[None, :]
        for k in range(len(m1)):
            m4 = -(m1[k] + s23)
            sh = geometry.shell_of_m2((m4 * m4).sum(-1), w, n_s)
            sel = sh == int(a4)
            if not sel.any():
                continue
            acc += v1[k] * np.sum(v23[sel] * val(m4[sel]))
            cnt += int(sel.sum())
        nq[t] = cnt
        with np.errstate(invalid="ignore", divide="ignore"):
            T[t] = acc.real / (vol * cnt)
            T_im[t] = acc.imag / (vol * cnt)
    return dict(T4=T, T4_imag=T_im, nquad=nq)
