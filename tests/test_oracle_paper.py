"""The oracle against values the paper prints (tests/golden/paper_printed_values.json)."""
import itertools
import json
import math
import os

import numpy as np
import pytest

from oracle import analytic, fbe, geometry

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.json")))


def test_bin_combination_counts():
    """Section 2.1: 15 rings give C(17,3) = 680 multisets, 120 at the largest k1, 105 at the next."""
    g = GOLD["binning_example"]
    n = g["n_rings"]
    multisets = list(itertools.combinations_with_replacement(range(1, n + 1), 3))
    assert len(multisets) == g["n_combinations_all"]
    assert sum(1 for c in multisets if max(c) == n) == g["n_combinations_largest_k1"]
    assert sum(1 for c in multisets if max(c) == n - 1) == g["n_combinations_second_k1"]
    # the oracle's closable subset is a subset of those and matches an independent enumeration
    ours = {tuple(r) for r in geometry.all_triangles(n)}
    brute = {tuple(sorted(c, reverse=True)) for c in multisets
             if sorted(c)[0] + sorted(c)[1] >= sorted(c)[2]}
    assert ours == brute


def test_shell_geometry_matches_printed_scales():
    """dk = 2 grid spacings = 0.0584 Mpc^-1 at L = 215 Mpc; largest (15th) shell centred at 0.88."""
    g = GOLD["binning_example"]
    kf = 2 * math.pi / g["box_l_mpc"]
    assert abs(g["dk_in_grid_spacings"] * kf - g["dk_mpc"]) < 5e-4
    _, means = geometry.shell_stats(2.0, 15)
    assert abs(means[14] * kf - g["k1_largest_ring_mpc"]) < 0.005
    assert abs(means[13] * kf - g["k1_second_ring_mpc"]) < 0.005


def test_cutoff_value():
    """Section 2.2: 2 pi N_g / (3 L) = 3.74 Mpc^-1 for N_g = 384, L = 215 Mpc."""
    c = GOLD["cutoff"]
    assert abs(2 * math.pi * c["n_g"] / (c["polyspectrum_order_p"] * c["box_l_mpc"]) - c["k_cut_mpc"]) < 0.005
    # the oracle's integer form of the rule: (n_s + 1/2) w <= N_g/3
    assert geometry.check_cutoff(24, 1.0, 7) and not geometry.check_cutoff(24, 1.0, 8)


def test_shell_mode_counts_small():
    """Shell 1 (w = 1) = |m|^2 in {1, 2}: 6 + 12 = 18 modes; shell 2 = |m|^2 in {3..6}: 8 + 6 + 24 + 24 = 62."""
    counts, _ = geometry.shell_stats(1.0, 3)
    r3 = {}
    for m in itertools.product(range(-3, 4), repeat=3):
        q = sum(c * c for c in m)
        r3[q] = r3.get(q, 0) + 1
    assert counts[0] == r3[1] + r3[2] == 18
    assert counts[1] == r3[3] + r3[4] + r3[5] + r3[6] == 62


def _lab(w, n_s, tri):
    _, means = geometry.shell_stats(w, n_s)
    k1, mu, t = geometry.labels(np.array([tri]), means)
    return float(mu[0]), float(t[0])


def test_printed_labels_dk2():
    g = GOLD["labels_dk2"]
    mu, t = _lab(2.0, 15, (15, 15, 1))
    assert t == 1.0 and round(mu, 3) == g["squeezed_mu"]
    mu, t = _lab(2.0, 15, (15, 15, 14))
    assert t == 1.0 and round(mu, 2) == g["near_equilateral_mu"]
    mu, t = _lab(2.0, 15, (15, 9, 6))
    assert (round(mu, 2), round(t, 2)) == tuple(g["stretched_like"])
    for tri in [(15, 14, 1), (15, 14, 2), (15, 15, 2)]:
        mu, t = _lab(2.0, 15, tri)
        assert mu >= g["near_squeezed_mu_min"] and t >= g["near_squeezed_t_min"]
    mu, t = _lab(2.0, 15, (15, 11, 10))
    assert round(t, 2) == g["cut_t"] and abs(mu - g["cut_mu_right_angle"]) < 0.01
    # the squeezed bin is the largest-mu bin at t = 1 for k1 = shell 15
    mus = [_lab(2.0, 15, (15, 15, a3))[0] for a3 in range(1, 16)]
    assert max(mus) == mus[0]


def test_printed_labels_dk1():
    g = GOLD["labels_dk1"]
    mu, t = _lab(1.0, 30, (30, 30, 29))
    assert t == 1.0 and round(mu, 2) == g["near_equilateral_mu"]
    mu, _ = _lab(1.0, 30, (30, 30, 2))
    assert round(mu, 3) == g["next_squeezed_mu"]
    mu, _ = _lab(1.0, 30, (30, 30, 1))
    # printed 0.9992; 3D shell means give 0.99910 (2D ring means 0.99919)
    assert abs(mu - g["squeezed_mu"]) < 2e-4


def test_ntri_claims_3d():
    """Section 3: N_tri ~ 1e7 for equilateral bins at k1 = shell 15 (dk = 2 k_f), falling by
    ~2 for right-angled and ~10 for linear triangles.  Geometry only, so N_g = 96 suffices."""
    g = GOLD["ntri_3d"]
    mask = fbe.shell_masks(96, 2.0, [1, 4, 10, 11, 15])
    I = {n: fbe.unit_field(m) for n, m in mask.items()}

    def ntri(a, b, c):
        return round(float(np.sum(I[a] * I[b] * I[c])) / 96 ** 3)
    eq = ntri(15, 15, 15)
    right = ntri(15, 11, 10)       # mu ~ t ~ 0.74 (the right-angle diagonal mu = t)
    linear = ntri(15, 11, 4)       # mu ~ 1
    assert 0.3 * g["equilateral_order"] < eq < 3 * g["equilateral_order"]
    assert 0.7 * g["right_angle_drop"] < eq / right < 1.5 * g["right_angle_drop"]
    assert 0.5 * g["linear_drop"] < eq / linear < 2.0 * g["linear_drop"]
    mu, t = _lab(2.0, 15, (15, 11, 10))
    assert abs(mu - t) < 0.02
    mu, _ = _lab(2.0, 15, (15, 11, 4))
    assert mu > 0.99


def test_rsd_monopole_closed_form_vs_monte_carlo():
    for sides in [(1.0, 1.0, 1.0), (1.0, 0.73, 0.69), (1.0, 1.0, 0.2), (1.0, 0.6, 0.45)]:
        r = analytic.rsd_monopole_factor(*sides, 1.0)
        m, err = analytic.rsd_monopole_factor_mc(*sides, 1.0, n_dirs=400000, seed=1)
        assert abs(r - m) < 5 * err
    # beta -> 0 limit and the equilateral closed value
    assert analytic.rsd_monopole_factor(1.0, 1.0, 1.0, 0.0) == 1.0
    assert abs(analytic.rsd_monopole_factor(1.0, 1.0, 1.0, 1.0) - (2.0 + 4.5 / 15 + 1.5 / 105)) < 1e-14


def test_rsd_enhancement_against_printed():
    """Section 3.1: printed B^s/B factors agree with the prediction within about 7 per cent."""
    g = GOLD["rsd_enhancement"]
    _, means = geometry.shell_stats(2.0, 15)
    cases = {"equilateral": (15, 15, 15), "t1_mu1": (15, 15, 1),
             "t073_mu074": (15, 11, 10), "t073_mu1": (15, 11, 4)}
    for key, tri in cases.items():
        k = [means[a - 1] for a in tri]
        r = analytic.rsd_monopole_factor(*k, g["beta"])
        assert abs(r / g[key] - 1.0) < g["agreement"], (key, r, g[key])
