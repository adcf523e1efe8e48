"""Shell geometry, triangle selection and bin labels (FP64, numpy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions (Section 2.1 of the paper; the readings are listed in the design notes):
  * k = k_f m with k_f = 2 pi / L and integer lattice vectors m.
  * Shells have uniform width dk = w k_f (w >= 1, since the paper finds widths
    below one grid spacing meaningless).  Shell n (n = 1..n_s) is centred on
    n dk and holds the modes with (n - 1/2) w <= |m| < (n + 1/2) w.  Membership
    is decided on the integer |m|^2: (2n-1)^2 w^2 <= 4|m|^2 < (2n+1)^2 w^2,
    evaluated in float64 exactly as written.
  * A triangle bin is a multiset of shells a1 >= a2 >= a3 (the paper counts
    C(17,3) = 680 such combinations for 15 rings); it can close only if
    a2 + a3 >= a1.
  * Labels (eq. shape): with k_n the mean |k| of the modes of shell n,
    t = k2/k1 and mu = (k1/k2 + k2/k1 - k3^2/(k1 k2))/2.
  * Aliasing cutoff (Section 2.2, eq. 3FT): every used mode must satisfy
    k < 2 pi N_g / (3 L), i.e. (n_s + 1/2) w <= N_g / 3.
"""
from __future__ import annotations

import math

import numpy as np

TRI_ALL, TRI_K1SET, TRI_MUT_GRID, TRI_LIST = 0, 1, 2, 3


def shell_of_m2(m2: np.ndarray, w: float, n_shells: int) -> np.ndarray:
    """Shell index (1..n_shells) of each integer |m|^2, 0 where outside every shell."""
    m2 = np.asarray(m2)
    four_m2 = 4.0 * m2.astype(np.float64)
    out = np.zeros(m2.shape, dtype=np.int32)
    ww = w * w
    for n in range(1, n_shells + 1):
        lo = float((2 * n - 1) ** 2) * ww
        hi = float((2 * n + 1) ** 2) * ww
        out[(four_m2 >= lo) & (four_m2 < hi)] = n
    return out


def check_cutoff(n_g: int, w: float, n_shells: int) -> bool:
    """True when every shell mode lies below 2 pi N_g/(3 L): (n_s + 1/2) w <= N_g/3."""
    return (n_shells + 0.5) * w * 3.0 <= n_g


def lattice_ball(radius: float) -> np.ndarray:
    """All integer vectors with |m| <= radius, shape (M, 3) int64."""
    r = int(math.ceil(radius))
    ax = np.arange(-r, r + 1)
    g = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), axis=-1).reshape(-1, 3)
    return g[(g * g).sum(1) <= radius * radius]


def shell_stats(w: float, n_shells: int):
    """(counts[n_s], mean_abs_m[n_s]) over the full 3D lattice (both k and -k)."""
    pts = lattice_ball((n_shells + 0.5) * w + 1.0)
    m2 = (pts * pts).sum(1)
    s = shell_of_m2(m2, w, n_shells)
    counts = np.zeros(n_shells, dtype=np.int64)
    means = np.zeros(n_shells, dtype=np.float64)
    absm = np.sqrt(m2.astype(np.float64))
    for n in range(1, n_shells + 1):
        sel = s == n
        counts[n - 1] = int(sel.sum())
        means[n - 1] = absm[sel].mean() if counts[n - 1] else float("nan")
    return counts, means


def all_triangles(n_shells: int, k1_set=None) -> np.ndarray:
    """All closable shell triples a1 >= a2 >= a3 >= 1 with a2 + a3 >= a1,
    ascending in (a1, a2, a3); optionally only a1 in k1_set.  int32 (T, 3)."""
    keep = None if k1_set is None else set(int(a) for a in k1_set)
    rows = []
    for a1 in range(1, n_shells + 1):
        if keep is not None and a1 not in keep:
            continue
        for a2 in range(1, a1 + 1):
            for a3 in range(1, a2 + 1):
                if a2 + a3 >= a1:
                    rows.append((a1, a2, a3))
    return np.array(rows, dtype=np.int32).reshape(-1, 3)


def grid_triangles(k1_shells, n_mu: int, n_t: int):
    """Shape-grid selection: for each k1 shell a1 and each point of the
    (mu, t) grid linspace(0.5, 1, n_mu) x linspace(0.5, 1, n_t) inside the
    domain t*mu >= 1/2 (eq. cond), the nearest shell triple
      a2 = clamp(floor(t a1 + 1/2), 1, a1)
      a3 = clamp(floor(a1 sqrt(1 + t^2 - 2 mu t) + 1/2), 1, a2)
    (k3 = -(k1 + k2) and mu = -k1.k2/(k1 k2) give
    |k3|^2 = k1^2 + k2^2 - 2 mu k1 k2, i.e. k3 = k1 sqrt(1 + t^2 - 2 mu t)).
    Returns (unique closable triples ascending, per-grid-point rows:
    (a1, mu, t, triangle index or -1))."""
    mus = np.linspace(0.5, 1.0, n_mu)
    ts = np.linspace(0.5, 1.0, n_t)
    picks = []
    for a1 in k1_shells:
        for t in ts:
            for mu in mus:
                if t * mu < 0.5 - 1e-12:
                    continue
                a2 = min(max(int(math.floor(t * a1 + 0.5)), 1), a1)
                a3 = int(math.floor(a1 * math.sqrt(max(0.0, 1.0 + t * t - 2.0 * mu * t)) + 0.5))
                a3 = min(max(a3, 1), a2)
                picks.append((int(a1), float(mu), float(t), a2, a3))
    uniq = sorted({(a1, a2, a3) for (a1, _, _, a2, a3) in picks if a2 + a3 >= a1})
    index = {tri: i for i, tri in enumerate(uniq)}
    grid = [(a1, mu, t, index.get((a1, a2, a3), -1)) for (a1, mu, t, a2, a3) in picks]
    return np.array(uniq, dtype=np.int32).reshape(-1, 3), grid


def labels(tri: np.ndarray, kmean: np.ndarray):
    """(k1, mu, t) per eq. shape from shell mean lengths kmean[n-1] (any unit)."""
    tri = np.asarray(tri)
    k1 = kmean[tri[:, 0] - 1]
    k2 = kmean[tri[:, 1] - 1]
    k3 = kmean[tri[:, 2] - 1]
    t = k2 / k1
    mu = 0.5 * (k1 / k2 + k2 / k1 - (k3 / k1) * (k3 / k2))
    return k1, mu, t
