"""The fourth-order polyspectrum (Section 4, p = 4) through the C ABI against
the float64 oracle (oracle/polyspectrum.py, itself pinned to the closed
4-tuple sum): N_quad exact; T with e_norm and max e_cond <= 1e-5 (e_cond over
the summation scale S = sum_x |D D D D| in the same normalisation)."""
import numpy as np
import pytest

from gpu_util import gpu_ok, metrics, say, to_gpu
from oracle import polyspectrum as poly
from synth import PowerLaw, gaussian_field, quadratic_ng_field

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ok(), reason="needs a GPU")]

TOL = 1e-5


def _field(n_g, box, seed):
    return quadratic_ng_field(gaussian_field(n_g, box, PowerLaw(-1.0), seed), 1.0)


def _check(plan, d64, box, dk, beta, idx=None):
    got = plan.run_last
    quads = plan.triangles.numpy()
    if idx is not None:
        quads, got = quads[idx], got[idx]
    ref = poly.fft_estimate(d64, box, dk, quads, rsd_beta=beta, with_abs=True)
    ntri = plan.ntri.numpy() if idx is None else plan.ntri.numpy()[idx]
    assert np.array_equal(ntri, ref["nquad"])
    m = metrics(got, ref["T4"], ref["S"])
    say("  n_g=%d n_quad=%d %s" % (d64.shape[0], len(quads), m))
    assert m["e_norm"] <= TOL and m["e_cond"] <= TOL, m
    return m


@pytest.mark.parametrize("n_g,box,dk,n_s,beta,extra", [
    (16, 100.0, 1.0, 3, 0.0, {}),
    (48, 200.0, 1.0, 10, 0.5, {}),                                # 651 bins, G = 48
    (64, 300.0, 1.5, 10, 1.0, {"tri_mode": 1, "k1_shells": [10, 7]}),
    (96, 400.0, 1.0, 20, 0.0, {"tri_mode": 3, "triangles": [(20, 20, 20, 20), (20, 10, 6, 4), (17, 9, 5, 3),
                                                          (12, 12, 1, 1), (1, 1, 1, 1), (20, 7, 7, 6)]}),
])
def test_order4_matches_oracle(n_g, box, dk, n_s, beta, extra):
    import torch
    import paper_2107_14564_amd as P
    dg, d64 = to_gpu(_field(n_g, box, 440 + n_g))
    plan = P.Plan(n_g, box, dk, n_s, rsd_beta=beta, order=4, **extra)
    plan.run_last = plan.run(dg).cpu().numpy()
    say("order 4: n_g=%d n_s=%d G=%d bins=%d" % (n_g, n_s, plan.n_est, plan.n_tri))
    _check(plan, d64, box, dk, beta)
    plan.close()


@pytest.mark.timeout(600)
def test_order4_thirty_shells_sampled():
    """N_g = 128 (L = 600 Mpc), 30 shells: all 35 345 bins on the GPU; 400 of
    them, spread over the bins, against the oracle on the full grid."""
    import paper_2107_14564_amd as P
    n_g, box = 128, 600.0
    dg, d64 = to_gpu(_field(n_g, box, 4128))
    plan = P.Plan(n_g, box, 1.0, 30, rsd_beta=0.5, order=4)
    plan.run_last = plan.run(dg).cpu().numpy()
    assert plan.n_tri == 35345 and plan.n_est == 128
    idx = np.unique(np.linspace(0, plan.n_tri - 1, 400).astype(int))
    _check(plan, d64, box, 1.0, 0.5, idx)
    plan.close()


def test_order4_kronecker_delta():
    """delta = Kronecker at the origin: Delta = dV for every mode, so T = dV^4 / V
    in every bin.  The shell fields cancel heavily here (sum |D D D D| is many
    times T), so the bound is the conditioned one, against the oracle's
    summation scale S."""
    import torch
    import paper_2107_14564_amd as P
    n_g, box = 48, 200.0
    d = np.zeros((n_g,) * 3, dtype=np.float32)
    d[0, 0, 0] = 1.0
    plan = P.Plan(n_g, box, 1.0, 10, order=4)
    t = plan.run(torch.from_numpy(d).cuda()).cpu().numpy()
    exact = (box / n_g) ** 12 / box ** 3
    ref = poly.fft_estimate(d.astype(np.float64), box, 1.0, plan.triangles.numpy(), with_abs=True)
    assert np.max(np.abs(ref["T4"] / exact - 1.0)) < 1e-10
    e_cond = float(np.max(np.abs(t - exact) / ref["S"]))
    say("  kronecker: e_cond=%.3g, max |T/exact - 1|=%.3g, S/T up to %.1f" % (
        e_cond, np.max(np.abs(t / exact - 1.0)), np.max(ref["S"] / exact)))
    assert e_cond <= TOL
    plan.close()


def test_order4_rejections():
    import paper_2107_14564_amd as P
    with pytest.raises(P.BispecError):     # the p = 4 cutoff: (12 + 1/2) x 4 > 48
        P.Plan(48, 200.0, 1.0, 12, order=4)
    with pytest.raises(P.BispecError):
        P.Plan(48, 200.0, 1.0, 10, order=4, precision=P.PREC_FP32)
    with pytest.raises(P.BispecError):
        P.Plan(48, 200.0, 1.0, 10, order=4, flags=P.FLAG_GRAD)
