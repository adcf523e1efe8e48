"""Seeded synthetic density fields of the kind the paper validates on.

The paper's validation field (Section 3, eq. nG) is a Gaussian random field
delta_G with a power-law power spectrum P(k) = A k^n, turned non-Gaussian by a
local quadratic term: delta = delta_G + f_NG (delta_G^2 - <delta_G^2>).

Recipe (the input recipe used by every test and by the benchmark):
  * white noise w(x) ~ N(0, 1) on the N^3 grid from numpy.random.default_rng(seed);
  * its unnormalised DFT W(k) has <|W|^2> = N^3, Hermitian symmetry and real
    self-conjugate modes by construction;
  * Delta_G(k) = W(k) sqrt(P(k) V / N^3), so that <|Delta_G|^2> = V P(k) with
    Delta(k) = dV * sum_x delta(x) exp(-i k.x) (the Fourier convention under
    which the paper's definition B = <Delta Delta Delta>/V holds);
    P(0) := 0;
  * delta_G = IDFT(Delta_G / dV) (numpy's normalised inverse);
  * <delta_G^2> is taken as the box mean.

Wave numbers are k = (2 pi / L) m with integer m in FFT order, in Mpc^-1 when L
is in Mpc.  Everything is float64; callers cast to float32 for the GPU and
give the oracle the same float32-rounded values.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

try:  # scipy's FFT is multi-threaded; numpy's is the fallback
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


@dataclasses.dataclass(frozen=True)
class PowerLaw:
    """P(k) = amplitude * k**index, with P(0) = 0."""
    index: float
    amplitude: float = 1.0

    def __call__(self, k: np.ndarray) -> np.ndarray:
        k = np.asarray(k, dtype=np.float64)
        out = np.zeros_like(k)
        nz = k > 0
        out[nz] = self.amplitude * k[nz] ** self.index
        return out


def _half_spectrum_k(n_g: int, box_l: float) -> np.ndarray:
    kf = 2.0 * math.pi / box_l
    m = np.fft.fftfreq(n_g, d=1.0 / n_g)
    mz = np.arange(n_g // 2 + 1, dtype=np.float64)
    k2 = (m[:, None, None] ** 2 + m[None, :, None] ** 2) + mz[None, None, :] ** 2
    return kf * np.sqrt(k2)


def gaussian_field(n_g: int, box_l: float, power: PowerLaw, seed: int) -> np.ndarray:
    """Seeded Gaussian random field delta_G(x), float64 [N][N][N] (z fastest)."""
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((n_g, n_g, n_g))
    vol = box_l ** 3
    dv = vol / n_g ** 3
    w_k = _rfftn(white)
    del white
    amp = np.sqrt(power(_half_spectrum_k(n_g, box_l)) * vol / n_g ** 3)
    w_k *= amp
    del amp
    w_k /= dv
    return _irfftn(w_k, s=(n_g, n_g, n_g))


def quadratic_ng_field(delta_g: np.ndarray, f_ng: float) -> np.ndarray:
    """delta = delta_G + f_NG (delta_G^2 - <delta_G^2>) with the box mean."""
    sq = delta_g * delta_g
    return delta_g + f_ng * (sq - sq.mean())


# The benchmark and parity workloads, as (N_g, L [Mpc], P(k), f_NG, seed).
WORKLOADS = {
    # oracle-sized case: N_g=32, L=300 Mpc, P = k^-1, f_NG = 1
    "ng32": dict(n_g=32, box_l=300.0, power=PowerLaw(-1.0), f_ng=1.0, seed=1001),
    # FP32 GPU case: N_g=256, L=1000 Mpc, P = k^-1, f_NG = 1
    "ng256": dict(n_g=256, box_l=1000.0, power=PowerLaw(-1.0), f_ng=1.0, seed=2001),
    # precision case: N_g=512, L=1500 Mpc, P = k^-1.5, f_NG = 2 (RSD beta=0.5 applied by the estimator)
    "ng512": dict(n_g=512, box_l=1500.0, power=PowerLaw(-1.5), f_ng=2.0, seed=3001),
    # the precision case on the smallest grid that holds its 100 shells: N_g=320, L=937.5 Mpc (same cell size)
    "ng320": dict(n_g=320, box_l=937.5, power=PowerLaw(-1.5), f_ng=2.0, seed=3003),
    # the precision case on the paper's largest grid: N_g=1024, L=3000 Mpc (the same cell size)
    "ng1024": dict(n_g=1024, box_l=3000.0, power=PowerLaw(-1.5), f_ng=2.0, seed=3002),
    # fourth-order case: N_g=128, L=600 Mpc, P = k^-1, f_NG = 1
    "ng128": dict(n_g=128, box_l=600.0, power=PowerLaw(-1.0), f_ng=1.0, seed=4128),
    # differentiation case: N_g=256, L=1000 Mpc, P = k^-1, f_NG = 1
    "ng256_grad": dict(n_g=256, box_l=1000.0, power=PowerLaw(-1.0), f_ng=1.0, seed=5001),
}


def workload_field(name: str, n_g: int | None = None, seed: int | None = None) -> np.ndarray:
    """The non-Gaussian field of a named workload (float64).  `n_g`/`seed`
    override the workload's grid size / seed (same box and spectrum)."""
    w = dict(WORKLOADS[name])
    if n_g is not None:
        w["n_g"] = n_g
    if seed is not None:
        w["seed"] = seed
    dg = gaussian_field(w["n_g"], w["box_l"], w["power"], w["seed"])
    return quadratic_ng_field(dg, w["f_ng"])


def batch_members(n: int = 64, seed: int = 4999, grids=(96, 128, 160), n_s_range=(16, 48),
                  box_l: float = 1000.0) -> list:
    """An ensemble of heterogeneous realisations (the batched form): per member
    N_g ~ U(grids), n_shells ~ U{n_s_range} clipped to the largest count below
    the aliasing cutoff at that N_g (shell width one k_f), f_NG ~ U(0.5, 2),
    P = k^-1, seed 4000 + i; the draws come from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        n_g = int(rng.choice(grids))
        n_s = int(rng.integers(n_s_range[0], n_s_range[1] + 1))
        n_s = min(n_s, int(np.floor(n_g / 3.0 - 0.5)))
        f_ng = float(rng.uniform(0.5, 2.0))
        out.append(dict(n_g=n_g, n_shells=n_s, f_ng=f_ng, seed=4000 + i, box_l=box_l))
    return out


def batch_field(member: dict) -> np.ndarray:
    """The non-Gaussian field of one batch member (float64)."""
    dg = gaussian_field(member["n_g"], member["box_l"], PowerLaw(-1.0), member["seed"])
    return quadratic_ng_field(dg, member["f_ng"])
