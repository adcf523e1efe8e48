"""Pins of the multipole oracle (oracle/multipoles.py) against what the
definition and the lattice fix, independently of its grid-sum code:
  - the weighted closed-triangle sum written out (brute force, 16^3);
  - l = 0 is the monopole estimator (eq. bsfin) exactly;
  - a Kronecker delta (Delta = dV for every mode): the closed triangles of any
    bin form a set invariant under permutations of the axes, so the mean of
    mu_1^2 over them is 1/3 and B_2 = 0 exactly;
  - a field that varies only along z has modes only on the z axis, so every
    closed triangle has mu_1 = +-1 and B_l = (2 l + 1) B_0; the same field
    along x has mu_1 = 0 and B_l = (2 l + 1) L_l(0) B_0 (L_2(0) = -1/2,
    L_4(0) = 3/8): this fixes the line of sight, the polynomials and the
    (2 l + 1) factor."""
import numpy as np
import pytest

from oracle import fbe, geometry, multipoles as mp
from synth import PowerLaw, gaussian_field, quadratic_ng_field


def _field(n_g, box, seed):
    return quadratic_ng_field(gaussian_field(n_g, box, PowerLaw(-1.0), seed), 1.0)


@pytest.mark.parametrize("ell,beta", [(2, 0.0), (2, 0.7), (4, 0.0), (4, 0.7)])
def test_grid_sum_equals_weighted_closed_sum(ell, beta):
    n_g, box, w = 16, 100.0, 1.0
    d = _field(n_g, box, 71 + ell)
    tri = geometry.all_triangles(4)
    fast = mp.estimate(d, box, w, tri, ell, rsd_beta=beta)
    slow = mp.direct_estimate(d, box, w, tri, ell, rsd_beta=beta)
    assert np.array_equal(fast["ntri"], slow["ntri"])
    scale = np.max(np.abs(slow["B"]))
    assert np.max(np.abs(fast["B"] - slow["B"])) <= 1e-10 * scale
    assert np.max(np.abs(slow["B_imag"])) <= 1e-10 * scale


def test_monopole_is_the_bispectrum():
    n_g, box = 32, 300.0
    d = _field(n_g, box, 5)
    tri = geometry.all_triangles(8)
    b0 = mp.estimate(d, box, 1.0, tri, 0, rsd_beta=0.5)["B"]
    b = fbe.estimate(d, box, 1.0, tri, rsd_beta=0.5)["B"]
    assert np.max(np.abs(b0 - b)) <= 1e-13 * np.max(np.abs(b))


def test_kronecker_quadrupole_vanishes():
    n_g, box = 32, 200.0
    d = np.zeros((n_g,) * 3)
    d[0, 0, 0] = 1.0
    tri = geometry.all_triangles(8)
    dv = (box / n_g) ** 3
    b0 = mp.estimate(d, box, 1.0, tri, 0)["B"]
    b2 = mp.estimate(d, box, 1.0, tri, 2)["B"]
    b4 = mp.estimate(d, box, 1.0, tri, 4)["B"]
    assert np.allclose(b0, dv ** 3 / box ** 3, rtol=1e-12)
    assert np.max(np.abs(b2)) <= 1e-12 * dv ** 3 / box ** 3
    # the hexadecapole is not fixed by the cubic symmetry: it must not vanish everywhere
    assert np.max(np.abs(b4)) > 1e-3 * dv ** 3 / box ** 3


@pytest.mark.parametrize("ell", [2, 4])
def test_axis_fields(ell):
    n_g, box = 32, 300.0
    rng = np.random.default_rng(9)
    z = np.arange(n_g) * 2 * np.pi / n_g
    prof = sum(rng.normal() * np.cos(m * z + rng.uniform(0, 2 * np.pi)) for m in range(1, 9))
    prof = prof + 0.3 * prof ** 2
    along_z = np.broadcast_to(prof[None, None, :], (n_g,) * 3).copy()
    along_x = np.broadcast_to(prof[:, None, None], (n_g,) * 3).copy()
    tri = np.array([t for t in geometry.all_triangles(8) if t[0] == t[1] + t[2]])  # collinear bins
    l0 = {2: -0.5, 4: 3.0 / 8.0}[ell]
    for field, factor in ((along_z, 2 * ell + 1), (along_x, (2 * ell + 1) * l0)):
        b0 = mp.estimate(field, box, 1.0, tri, 0)["B"]
        bl = mp.estimate(field, box, 1.0, tri, ell)["B"]
        big = np.abs(b0) > 1e-6 * np.max(np.abs(b0))
        assert big.sum() >= 5
        assert np.max(np.abs(bl[big] / (factor * b0[big]) - 1.0)) < 1e-9


def test_rejects_odd_orders():
    with pytest.raises(ValueError):
        mp.legendre(1, np.zeros(3))
