"""Legendre multipoles of the redshift-space bispectrum (ell = 2, 4) through
the C ABI against the float64 oracle (oracle/multipoles.py, pinned to the
weighted closed-triangle sum): N_tri exact, e_norm and max e_cond <= 1e-5
(e_cond over the oracle's summation scale S = (2 ell + 1) sum_x |D^l D D| /
(V N_tri N^3)); ell = 0 is bit for bit the bispectrum plan."""
import numpy as np
import pytest

from gpu_util import gpu_ok, metrics, say, to_gpu
from oracle import multipoles as mp
from synth import PowerLaw, gaussian_field, quadratic_ng_field

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ok(), reason="needs a GPU")]

TOL = 1e-5


def _field(n_g, box, seed):
    return quadratic_ng_field(gaussian_field(n_g, box, PowerLaw(-1.0), seed), 1.0)


def _check(plan, b, d64, box, dk, beta, ell, idx=None):
    tri = plan.triangles.numpy()
    ntri = plan.ntri.numpy()
    if idx is not None:
        tri, ntri, b = tri[idx], ntri[idx], b[idx]
    ref = mp.estimate(d64, box, dk, tri, ell, rsd_beta=beta, with_abs=True)
    assert np.array_equal(ntri, ref["ntri"])
    m = metrics(b, ref["B"], ref["S"])
    say("  ell=%d n_tri=%d %s" % (ell, len(tri), m))
    assert m["e_norm"] <= TOL and m["e_cond"] <= TOL, m


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("ell", [2, 4])
@pytest.mark.parametrize("n_g,box,dk,n_s,beta,extra", [
    (32, 300.0, 1.0, 10, 0.5, {}),
    (64, 300.0, 1.0, 20, 0.7, {}),                        # grid classes, replicated tilings
    (48, 200.0, 1.5, 9, 1.0, {"tri_mode": 1, "k1_shells": [9, 8, 5]}),
])
def test_multipole_matches_oracle(n_g, box, dk, n_s, beta, extra, ell, precision):
    import paper_2107_14564_amd as P
    dg, d64 = to_gpu(_field(n_g, box, 900 + n_g + ell))
    plan = P.Plan(n_g, box, dk, n_s, rsd_beta=beta, precision=precision, ell=ell, **extra)
    b = plan.run(dg).cpu().numpy()
    say("multipole ell=%d n_g=%d n_s=%d prec=%d classes %s" % (ell, n_g, n_s, precision, plan.class_grids))
    _check(plan, b, d64, box, dk, beta, ell)
    plan.close()


@pytest.mark.timeout(600)
def test_quadrupole_forty_shells_sampled():
    """N_g = 128, 40 shells, beta = 0.5 (several grid classes, up to 40 + 40
    staged rows): 300 bins spread over the selection against the oracle."""
    import paper_2107_14564_amd as P
    n_g, box = 128, 600.0
    dg, d64 = to_gpu(_field(n_g, box, 1280))
    plan = P.Plan(n_g, box, 1.0, 40, rsd_beta=0.5, ell=2)
    b = plan.run(dg).cpu().numpy()
    idx = np.unique(np.linspace(0, plan.n_tri - 1, 300).astype(int))
    _check(plan, b, d64, box, 1.0, 0.5, 2, idx)
    plan.close()


def test_monopole_plan_is_the_bispectrum_plan():
    import paper_2107_14564_amd as P
    dg, _ = to_gpu(_field(64, 300.0, 4))
    p0 = P.Plan(64, 300.0, 1.0, 20, rsd_beta=0.5, ell=0)
    pb = P.Plan(64, 300.0, 1.0, 20, rsd_beta=0.5)
    assert np.array_equal(p0.run(dg).cpu().numpy(), pb.run(dg).cpu().numpy())
    p0.close()
    pb.close()


def test_axis_field_factors():
    """A field varying only along z (x): every contributing triangle has
    mu_1 = +-1 (0), so B_l / B_0 = 2 l + 1 ((2 l + 1) L_l(0)) on the bins the
    field populates."""
    import torch
    import paper_2107_14564_amd as P
    n_g, box = 32, 300.0
    rng = np.random.default_rng(9)
    z = np.arange(n_g) * 2 * np.pi / n_g
    prof = sum(rng.normal() * np.cos(m * z + rng.uniform(0, 2 * np.pi)) for m in range(1, 9))
    prof = prof + 0.3 * prof ** 2
    tri = [(a, b, a - b) for a in range(2, 9) for b in range(1, a) if a - b <= b]
    for axis, l2, l4 in ((2, 1.0, 1.0), (0, -0.5, 3.0 / 8.0)):
        shape = [1, 1, 1]
        shape[axis] = n_g
        d = np.broadcast_to(prof.reshape(shape), (n_g,) * 3).astype(np.float32).copy()
        dg = torch.from_numpy(d).cuda()
        out = {}
        for ell in (0, 2, 4):
            plan = P.Plan(n_g, box, 1.0, 8, ell=ell, tri_mode=3, triangles=tri)
            out[ell] = plan.run(dg).cpu().numpy()
            plan.close()
        big = np.abs(out[0]) > 1e-3 * np.max(np.abs(out[0]))
        assert big.sum() >= 5
        for ell, lv in ((2, l2), (4, l4)):
            r = out[ell][big] / ((2 * ell + 1) * lv * out[0][big])
            say("  axis %d ell %d ratio range %g %g" % (axis, ell, r.min(), r.max()))
            assert np.max(np.abs(r - 1.0)) < 1e-4


def test_multipole_rejections():
    import paper_2107_14564_amd as P
    with pytest.raises(P.BispecError):
        P.Plan(32, 300.0, 1.0, 10, ell=3)
    with pytest.raises(P.BispecError):
        P.Plan(32, 300.0, 1.0, 10, ell=2, flags=P.FLAG_GRAD)
    with pytest.raises(P.BispecError):
        P.Plan(48, 200.0, 1.0, 10, ell=2, order=4)
