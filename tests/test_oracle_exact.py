"""The FP64 oracle against exact facts: the direct triple sum on small grids,
closed forms and exact invariances (CPU only)."""
import itertools

import numpy as np
import pytest

from oracle import adjoint, dbe, fbe, geometry
from synth import workload_field

L16 = 100.0


def _field(n_g, seed):
    return workload_field("ng32", n_g=n_g, seed=seed)


@pytest.mark.parametrize("w,n_s,beta", [(1.0, 4, 0.0), (1.0, 4, 0.5), (1.5, 3, 0.0), (2.0, 2, 1.0)])
def test_fbe_equals_direct_sum(w, n_s, beta):
    """eq. bsfin (FFT form) reproduces eq. binbs (direct form) exactly below the cutoff."""
    d = _field(16, 11)
    tri = geometry.all_triangles(n_s)
    a = fbe.estimate(d, L16, w, tri, rsd_beta=beta)
    b = dbe.estimate(d, L16, w, tri, rsd_beta=beta)
    assert np.array_equal(a["ntri"], b["ntri"])
    assert np.all(a["ntri"] > 0)
    assert a["ntri_resid"] < 1e-8
    np.testing.assert_allclose(a["B"], b["B"], rtol=1e-11, atol=0)
    assert np.max(np.abs(b["B_imag"]) / np.abs(b["B"])) < 1e-11


def test_direct_sum_tiny_grid_by_hand():
    """N_g = 8: shells 1, 2 (w = 1), checked against an explicit Python loop over mode triples."""
    d = _field(8, 5)
    L = 40.0
    tri = geometry.all_triangles(2)
    a = fbe.estimate(d, L, 1.0, tri)
    spec = np.fft.fftn(d) * (L / 8) ** 3
    modes = [m for m in itertools.product(range(-3, 4), repeat=3)]
    shell = {m: int(np.floor(np.sqrt(sum(c * c for c in m)) + 0.5)) for m in modes}
    for t, (a1, a2, a3) in enumerate(tri):
        tot, cnt = 0.0, 0
        for m1 in modes:
            if shell[m1] != a1 or sum(c * c for c in m1) == 0:
                continue
            for m2 in modes:
                if shell[m2] != a2 or sum(c * c for c in m2) == 0:
                    continue
                m3 = tuple(-x - y for x, y in zip(m1, m2))
                if m3 in shell and shell[m3] == a3 and sum(c * c for c in m3) > 0:
                    tot += (spec[m1] * spec[m2] * spec[m3]).real
                    cnt += 1
        assert cnt == a["ntri"][t]
        assert abs(tot / (L ** 3 * cnt) - a["B"][t]) <= 1e-11 * abs(a["B"][t])


def test_kronecker_delta_input():
    """delta = 1 at one voxel => Delta(k) = dV e^{-ik.x0} => B = dV^3 / V for every bin."""
    d = np.zeros((16, 16, 16))
    d[3, 5, 7] = 1.0
    tri = geometry.all_triangles(4)
    B = fbe.estimate(d, L16, 1.0, tri)["B"]
    dv = (L16 / 16) ** 3
    np.testing.assert_allclose(B, dv ** 3 / L16 ** 3, rtol=1e-12)


def test_invariances():
    d = _field(16, 3)
    tri = geometry.all_triangles(4)
    base = fbe.estimate(d, L16, 1.0, tri, rsd_beta=0.5)["B"]
    # circular translation
    sh = fbe.estimate(np.roll(d, (3, -5, 2), axis=(0, 1, 2)), L16, 1.0, tri, rsd_beta=0.5)["B"]
    np.testing.assert_allclose(sh, base, rtol=1e-10)
    # x <-> y swap keeps the line of sight (z): exact symmetry with RSD
    sw = fbe.estimate(np.swapaxes(d, 0, 1).copy(), L16, 1.0, tri, rsd_beta=0.5)["B"]
    np.testing.assert_allclose(sw, base, rtol=1e-10)
    # inversion x -> -x maps Delta(k) -> Delta(k)^*, which leaves the real B unchanged
    inv = fbe.estimate(np.roll(d[::-1, ::-1, ::-1], 1, axis=(0, 1, 2)), L16, 1.0, tri, rsd_beta=0.5)["B"]
    np.testing.assert_allclose(inv, base, rtol=1e-10)
    # sign flip of the field flips B
    neg = fbe.estimate(-d, L16, 1.0, tri, rsd_beta=0.5)["B"]
    np.testing.assert_allclose(neg, -base, rtol=1e-12)
    # homogeneity of degree 3
    sc = fbe.estimate(2.5 * d, L16, 1.0, tri, rsd_beta=0.5)["B"]
    np.testing.assert_allclose(sc, 2.5 ** 3 * base, rtol=1e-12)


def test_rsd_breaks_z_swap_symmetry():
    """With RSD, swapping x <-> z is not a symmetry (the line of sight is z)."""
    d = _field(16, 4)
    tri = geometry.all_triangles(3)
    b0 = fbe.estimate(d, L16, 1.0, tri, rsd_beta=1.0)["B"]
    b1 = fbe.estimate(np.swapaxes(d, 0, 2).copy(), L16, 1.0, tri, rsd_beta=1.0)["B"]
    assert np.max(np.abs(b0 - b1) / np.abs(b0)) > 1e-3
    c0 = fbe.estimate(d, L16, 1.0, tri)["B"]
    c1 = fbe.estimate(np.swapaxes(d, 0, 2).copy(), L16, 1.0, tri)["B"]
    np.testing.assert_allclose(c0, c1, rtol=1e-10)


@pytest.mark.parametrize("beta", [0.0, 0.5])
def test_adjoint_equals_direct_gradient(beta):
    d = _field(16, 9)
    tri = geometry.all_triangles(4)
    v = np.random.default_rng(2).standard_normal(len(tri))
    g1 = adjoint.gradient(d, L16, 1.0, tri, v, rsd_beta=beta)
    g2 = dbe.gradient(d, L16, 1.0, tri, v, rsd_beta=beta)
    assert np.max(np.abs(g1 - g2)) <= 1e-11 * np.max(np.abs(g2))


def test_adjoint_finite_differences():
    d = _field(16, 10)
    tri = geometry.all_triangles(4)
    v = np.random.default_rng(5).standard_normal(len(tri))
    g = adjoint.gradient(d, L16, 1.0, tri, v, rsd_beta=0.5)
    rng = np.random.default_rng(6)
    h = 1e-4
    for _ in range(4):
        x = tuple(rng.integers(0, 16, 3))
        dp, dm = d.copy(), d.copy()
        dp[x] += h
        dm[x] -= h
        fd = (v @ fbe.estimate(dp, L16, 1.0, tri, 0.5)["B"] - v @ fbe.estimate(dm, L16, 1.0, tri, 0.5)["B"]) / (2 * h)
        assert abs(fd - g[x]) <= 1e-6 * np.max(np.abs(g))


def test_adjoint_dot_product():
    """<v, J u> = <J^T v, u> with J u from a directional finite difference of B."""
    d = _field(16, 12)
    tri = geometry.all_triangles(3)
    rng = np.random.default_rng(8)
    v = rng.standard_normal(len(tri))
    u = rng.standard_normal(d.shape)
    g = adjoint.gradient(d, L16, 1.0, tri, v)
    h = 1e-3

    def B(s):
        return fbe.estimate(d + s * u, L16, 1.0, tri)["B"]
    # B is a cubic polynomial in s: this five-point stencil is exact for degree <= 4
    ju = (8.0 * (B(h) - B(-h)) - (B(2 * h) - B(-2 * h))) / (12.0 * h)
    assert abs(v @ ju - np.sum(g * u)) <= 1e-9 * abs(v @ ju)


def test_aliasing_above_cutoff():
    """Section 2.2 (eq. 3FT): the FFT count equals the direct count while every mode
    is below 2 pi N_g/(3L) and exceeds it beyond (equilateral bins, N_g = 24, w = 1)."""
    d = np.zeros((24, 24, 24))
    ratios = {}
    for n in range(1, 12):
        tri = np.array([[n, n, n]])
        a = fbe.estimate(d, 50.0, 1.0, tri, enforce_cutoff=False)
        b = dbe.estimate(d, 50.0, 1.0, tri)
        ratios[n] = a["ntri"][0] / b["ntri"][0]
    for n in range(1, 8):          # top edge (n + 1/2) <= 8 = N_g/3
        assert ratios[n] == 1.0
    for n in range(8, 12):
        assert ratios[n] > 1.0
    assert ratios[11] > ratios[8]


def test_cutoff_enforced():
    d = np.zeros((24, 24, 24))
    with pytest.raises(ValueError):
        fbe.estimate(d, 50.0, 1.0, np.array([[8, 8, 8]]))


def test_field_on_another_grid_is_the_mode_sum():
    """shell_field_at evaluates D_n(x) = sum_{k in n} Delta(k) e^{ik.x} at the points
    of a coarser grid: against the explicit complex sum over the full spectrum at
    a few points, and equal to shell_field on the input grid itself."""
    n_g, L = 16, L16
    d = _field(n_g, 21)
    spec = fbe.spectrum(d, L, 0.5)
    masks = fbe.shell_masks(n_g, 1.0, [2, 3])
    full = np.fft.fftn(d) * (L / n_g) ** 3
    m = np.fft.fftfreq(n_g, d=1.0 / n_g)
    mx, my, mz = np.meshgrid(m, m, m, indexing="ij")
    m2 = mx ** 2 + my ** 2 + mz ** 2
    with np.errstate(invalid="ignore", divide="ignore"):
        z = np.where(m2 > 0, 1 + 0.5 * mz ** 2 / np.where(m2 > 0, m2, 1), 1.0)
    shell_full = geometry.shell_of_m2(m2.astype(np.int64), 1.0, 3)
    for n in (2, 3):
        np.testing.assert_allclose(fbe.shell_field_at(spec, masks[n], n_g), fbe.shell_field(spec, masks[n]),
                                   rtol=0, atol=1e-12 * np.abs(fbe.shell_field(spec, masks[n])).max())
        g = 12                                   # modes |m_i| <= 3 < 6
        coarse = fbe.shell_field_at(spec, masks[n], g)
        sel = shell_full == n
        for j in [(0, 0, 0), (1, 5, 11), (7, 3, 2), (11, 11, 6)]:
            phase = 2j * np.pi * (mx[sel] * j[0] + my[sel] * j[1] + mz[sel] * j[2]) / g
            ref = np.sum(z[sel] * full[sel] * np.exp(phase))
            assert abs(ref.imag) < 1e-9 * abs(ref.real) + 1e-12
            assert abs(coarse[j] - ref.real) <= 1e-10 * np.abs(coarse).max()
    with pytest.raises(ValueError):
        fbe.shell_field_at(spec, masks[3], 6)


def test_triple_sum_on_a_coarser_grid():
    """Section 2.2's aliasing argument on an evaluation grid G: the G^3-point sum of
    D_a1 D_a2 D_a3, scaled by (N/G)^3, equals the N^3-point sum when G > 3 max|m_i|
    (and counts extra triangles when G is smaller)."""
    n_g, L, n_s = 24, 50.0, 4        # shells 1-4, max component 4
    d = _field(n_g, 33)
    spec = fbe.spectrum(d, L)
    tri = geometry.all_triangles(n_s)
    masks = fbe.shell_masks(n_g, 1.0, list(range(1, n_s + 1)))
    ref = fbe.triple_sums({n: fbe.shell_field(spec, masks[n]) for n in masks}, tri)
    for g in (13, 16, 20):
        fields = {n: fbe.shell_field_at(spec, masks[n], g) for n in masks}
        got = fbe.triple_sums(fields, tri) * (n_g / g) ** 3
        np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())
    ones = {n: fbe.shell_field_at(masks[n].astype(np.complex128), masks[n], 12) for n in masks}
    n12 = fbe.triple_sums(ones, tri) / 12 ** 3
    exact = fbe.estimate(np.zeros((n_g,) * 3), L, 1.0, tri)["ntri"]
    assert np.any(np.rint(n12) > exact)       # G = 12 = 3 * 4 aliases
