"""The fourth-order polyspectrum oracle against the definitions it rests on.

Section 4 of the paper: the FFT form of the p-th order polyspectrum picks
exactly the closed p-tuples while every mode lies below 2 pi N_g / (p L).
Pins: the grid-sum form equals the closed-4-tuple sum written out (with and
without linear RSD) and counts the same N_quad; above the p = 4 cutoff (yet
below the bispectrum's p = 3 one) the grid sum counts aliased 4-tuples; a
Kronecker delta gives T = dV^4 / V in every bin; translations leave T
unchanged."""
import numpy as np
import pytest

from oracle import polyspectrum as poly
from synth import PowerLaw, gaussian_field, quadratic_ng_field

L16 = 100.0


def _field(n_g, seed):
    return quadratic_ng_field(gaussian_field(n_g, L16 * n_g / 16, PowerLaw(-1.0), seed), 1.0)


def test_all_quads_closable_counts():
    q = poly.all_quads(4)
    assert np.all(q[:, 0] >= q[:, 1]) and np.all(q[:, 1] >= q[:, 2]) and np.all(q[:, 2] >= q[:, 3])
    assert np.all(q[:, 1] + q[:, 2] + q[:, 3] >= q[:, 0])
    # multisets of 4 from 4 shells = C(7, 4) = 35; (4,1,1,1) cannot close
    assert len(q) == 34 and (4, 1, 1, 1) not in set(map(tuple, q.tolist()))


@pytest.mark.parametrize("beta", [0.0, 0.5])
def test_fft_form_equals_closed_quadrilateral_sum(beta):
    d = _field(16, 21)
    q = poly.all_quads(3)          # (3 + 1/2) x 4 = 14 <= 16
    f = poly.fft_estimate(d, L16, 1.0, q, rsd_beta=beta)
    b = poly.direct_estimate(d, L16, 1.0, q, rsd_beta=beta)
    assert np.array_equal(f["nquad"], b["nquad"]) and np.all(b["nquad"] > 0)
    assert np.max(np.abs(b["T4_imag"])) <= 1e-10 * np.max(np.abs(b["T4"]))
    np.testing.assert_allclose(f["T4"], b["T4"], rtol=1e-10, atol=1e-13 * np.max(np.abs(b["T4"])))


def test_cutoff_of_the_fourth_order():
    """At N_g = 12 with 3 shells, (3 + 1/2) x 3 = 10.5 <= 12 keeps the
    bispectrum exact but (3 + 1/2) x 4 = 14 > 12: the grid sum counts
    aliased 4-tuples for some bins."""
    d = _field(12, 22)
    q = poly.all_quads(3)
    f = poly.fft_estimate(d, 75.0, 1.0, q, enforce_cutoff=False)
    b = poly.direct_estimate(d, 75.0, 1.0, q)
    assert np.any(f["nquad"] > b["nquad"])
    assert np.all(f["nquad"] >= b["nquad"])
    with pytest.raises(ValueError):
        poly.fft_estimate(d, 75.0, 1.0, q)


def test_kronecker_delta_closed_form():
    n_g = 16
    d = np.zeros((n_g,) * 3)
    d[0, 0, 0] = 1.0
    q = poly.all_quads(3)
    f = poly.fft_estimate(d, L16, 1.0, q)
    dv = (L16 / n_g) ** 3
    np.testing.assert_allclose(f["T4"], dv ** 4 / L16 ** 3, rtol=1e-12)


def test_translation_invariance():
    d = _field(16, 23)
    q = poly.all_quads(3)
    a = poly.fft_estimate(d, L16, 1.0, q)["T4"]
    b = poly.fft_estimate(np.roll(d, (5, -3, 7), axis=(0, 1, 2)), L16, 1.0, q)["T4"]
    np.testing.assert_allclose(a, b, rtol=1e-10, atol=1e-13 * np.max(np.abs(a)))
