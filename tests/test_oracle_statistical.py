"""The oracle against the paper's analytic predictions, statistically.

eq. bana gives the tree-level bispectrum of delta = delta_G + f_NG q,
q = delta_G^2 - <delta_G^2>.  The estimator is a cubic form, so the
antisymmetrised combination [B(delta_G + f q) - B(delta_G - f q)] / (2 f)
keeps the part linear in f (whose mean is 2[P1P2 + P2P3 + P3P1], bin-averaged
as in eq. binavgbs) plus an f^2-suppressed cubic-in-q term, and cancels the
pure-Gaussian term that dominates the scatter of a single realisation."""
import numpy as np
import pytest

from oracle import analytic, fbe, geometry
from synth import PowerLaw, gaussian_field

N_G, BOX, W, N_S, F = 32, 300.0, 1.0, 10, 0.05
POWER = PowerLaw(-1.0)


def _ensemble(n_real, beta, tri):
    ys = []
    for r in range(n_real):
        dg = gaussian_field(N_G, BOX, POWER, seed=7000 + r)
        q = dg * dg - np.mean(dg * dg)
        bp = fbe.estimate(dg + F * q, BOX, W, tri, rsd_beta=beta)["B"]
        bm = fbe.estimate(dg - F * q, BOX, W, tri, rsd_beta=beta)["B"]
        ys.append((bp - bm) / (2 * F))
    ys = np.array(ys)
    return ys.mean(0), ys.std(0, ddof=1) / np.sqrt(n_real)


@pytest.mark.parametrize("beta", [0.0, 1.0])
def test_ensemble_mean_matches_bin_averaged_tree_level(beta):
    tri = geometry.all_triangles(N_S, k1_set=[7, 8, 9, 10])
    mean, err = _ensemble(48, beta, tri)
    pred = analytic.b_tree_binavg(N_G, BOX, W, tri, POWER, 1.0, rsd_beta=beta)
    z = (mean - pred) / err
    chi2 = float(np.mean(z * z))
    assert chi2 < 1.6, chi2
    assert np.max(np.abs(z)) < 5.0
    # the test has power: a 15 per cent error in the prediction is rejected
    z_bad = (mean - 1.15 * pred) / err
    assert float(np.mean(z_bad * z_bad)) > 3.0


def test_bin_average_approaches_label_value_for_thin_bins():
    """The bin-averaged prediction differs from eq. bana at the labels by a finite-width
    effect that is largest near the squeezed corner (Section 3's explanation)."""
    _, means = geometry.shell_stats(W, N_S)
    kf = 2 * np.pi / BOX
    tri = np.array([[10, 10, 10], [10, 9, 8], [10, 10, 1]])
    pred = analytic.b_tree_binavg(N_G, BOX, W, tri, POWER, 1.0)
    k = kf * means[tri - 1]
    at_labels = analytic.b_tree(k[:, 0], k[:, 1], k[:, 2], POWER, 1.0)
    rel = np.abs(pred / at_labels - 1)
    assert rel[0] < 0.05 and rel[1] < 0.05
    assert rel[2] > rel[0]


def test_gaussian_variance_matches_eq_cv():
    """The scatter of the estimated B of Gaussian fields against the Gaussian
    term of eq. cv, V <P1 P2 P3> / N_tri, bin-averaged, in bins of three
    distinct shells.  A variance estimate from n realisations has a relative
    spread of sqrt(2 / (n - 1)) per bin; averaged over the bins the ratio must
    be 1 within 12 %, and a formula off by a factor 2 (e.g. without the mirror
    pairing) is rejected."""
    tri = np.array([t for t in geometry.all_triangles(N_S, k1_set=[8, 9, 10]).tolist() if len(set(t)) == 3])
    n_real = 96
    bs = np.array([fbe.estimate(gaussian_field(N_G, BOX, POWER, seed=9100 + r), BOX, W, tri)["B"]
                   for r in range(n_real)])
    var_sim = bs.var(0, ddof=1)
    var_cv = analytic.gaussian_variance_binavg(N_G, BOX, W, tri, POWER)
    ratio = var_sim / var_cv
    assert abs(float(np.mean(ratio)) - 1.0) < 0.12, float(np.mean(ratio))
    assert float(np.median(ratio)) > 0.75 and float(np.median(ratio)) < 1.3
    assert abs(float(np.mean(var_sim / (2.0 * var_cv))) - 1.0) > 0.3
    with pytest.raises(ValueError):
        analytic.gaussian_variance_binavg(N_G, BOX, W, [[10, 10, 5]], POWER)
