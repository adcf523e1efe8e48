"""Parity at the full benchmark size (N_g = 512, L = 1500 Mpc, P = k^-1.5,
f_NG = 2, RSD beta = 0.5, 100 shells of one k_f, all 89 625 closable
triangles), in the launch configuration bench.py times.

The float64 oracle cannot hold all 100 shells at 512^3 on the host, so it is
evaluated one by one on a sample of triangles (all closable triangles among a
spread of shells); N_tri of the sample must be exact and B must meet the
1e-5 gate (normwise over the sample and conditioned per triangle)."""
import time

import numpy as np
import pytest

from gpu_util import gpu_ok, metrics, say, to_gpu
from oracle import fbe, geometry
from synth import workload_field

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ok(), reason="needs a GPU")]

SAMPLE_SHELLS = [1, 2, 3, 34, 50, 51, 99, 100]


@pytest.mark.timeout(900)
def test_fullsize_sampled_parity():
    import paper_2107_14564_amd as P
    n_g, box, dk, n_s, beta = 512, 1500.0, 1.0, 100, 0.5
    t0 = time.time()
    delta_gpu, delta64 = to_gpu(workload_field("ng512"))
    say("field %.1fs" % (time.time() - t0))
    plan = P.Plan(n_g, box, dk, n_s, rsd_beta=beta, precision=P.PREC_SPLITBF16)
    assert plan.n_tri == 89625
    b_split = plan.run(delta_gpu).cpu().numpy()
    plan.set_precision(P.PREC_FP32)
    b_fp32 = plan.run(delta_gpu).cpu().numpy()
    say("gpu done %.1fs; split vs fp32 normwise %.3g" % (time.time() - t0,
        np.linalg.norm(b_split - b_fp32) / np.linalg.norm(b_fp32)))
    tri_all = plan.triangles.numpy()
    ntri_all = plan.ntri.numpy()
    index = {tuple(r): t for t, r in enumerate(tri_all.tolist())}
    sset = set(SAMPLE_SHELLS)
    sample = [r for r in geometry.all_triangles(n_s).tolist() if set(r) <= sset]
    idx = np.array([index[tuple(r)] for r in sample])
    ref = fbe.estimate(delta64, box, dk, np.array(sample), rsd_beta=beta, with_abs=True)
    say("oracle %.1fs on %d triangles" % (time.time() - t0, len(sample)))
    assert np.array_equal(ntri_all[idx], ref["ntri"])
    cond = ref["S"] / np.abs(ref["B"])
    for name, b in (("fp32", b_fp32), ("split-bf16", b_split)):
        m = metrics(b[idx], ref["B"], ref["S"])
        say(name, m)
        rel = np.abs(b[idx] - ref["B"]) / np.abs(ref["B"])
        for k in np.argsort(-rel)[:5]:
            say("   worst %s B=%.6g ref=%.6g rel=%.3g cond=%.3g" % (sample[k], b[idx][k], ref["B"][k], rel[k],
                                                                      cond[k]))
        assert m["e_cond"] <= 1e-5 and m["e_norm"] <= 1e-5, (name, m)
    plan.close()


@pytest.mark.timeout(1100)
def test_ng1024_sampled_parity():
    """The same estimator on a 1024^3 grid (L = 3000 Mpc, the same cell size;
    the estimator grid stays G = 320): all closable triangles of shells 1 and
    100 -- the lowest and highest shell, (1,1,1), (100,100,1), (100,100,100) --
    against the float64 oracle on the full 1024^3 grid (about 80 GB of host
    memory for its fields)."""
    import paper_2107_14564_amd as P
    n_g, box, dk, n_s, beta = 1024, 3000.0, 1.0, 100, 0.5
    t0 = time.time()
    delta_gpu, delta64 = to_gpu(workload_field("ng1024"))
    say("field %.1fs" % (time.time() - t0))
    plan = P.Plan(n_g, box, dk, n_s, rsd_beta=beta, precision=P.PREC_SPLITBF16)
    assert plan.n_tri == 89625 and plan.n_est == 320
    b_split = plan.run(delta_gpu).cpu().numpy()
    tri_all = plan.triangles.numpy()
    ntri_all = plan.ntri.numpy()
    plan.close()
    del delta_gpu
    index = {tuple(r): t for t, r in enumerate(tri_all.tolist())}
    sample = [r for r in geometry.all_triangles(n_s).tolist() if set(r) <= {1, 100}]
    assert len(sample) == 3
    idx = np.array([index[tuple(r)] for r in sample])
    ref = fbe.estimate(delta64, box, dk, np.array(sample), rsd_beta=beta, with_abs=True)
    say("oracle %.1fs on %d triangles" % (time.time() - t0, len(sample)))
    assert np.array_equal(ntri_all[idx], ref["ntri"])
    m = metrics(b_split[idx], ref["B"], ref["S"])
    say("split-bf16", m)
    assert m["e_cond"] <= 1e-5 and m["e_norm"] <= 1e-5, m


@pytest.mark.timeout(900)
def test_max_shells_sampled_parity():
    """The largest split-bf16 plan: 128 shells of one k_f, which needs the
    estimator grid G = 512 (> 3 x 128), on the 512^3 benchmark field; the
    contraction's widest row sets (up to 128 shells staged per work group).
    All closable triangles among shells {1, 2, 64, 65, 127, 128} and two
    triangles of every wavefront slot shape of its tiling against the float64
    oracle, N_tri exact and the 1e-5 gate for both precisions."""
    import paper_2107_14564_amd as P
    n_g, box, dk, n_s, beta = 512, 1500.0, 1.0, 128, 0.5
    t0 = time.time()
    delta_gpu, delta64 = to_gpu(workload_field("ng512"))
    plan = P.Plan(n_g, box, dk, n_s, rsd_beta=beta, precision=P.PREC_SPLITBF16)
    say("plan %.1fs: G=%d n_tri=%d" % (time.time() - t0, plan.n_est, plan.n_tri))
    assert plan.n_est == 512
    b_split = plan.run(delta_gpu).cpu().numpy()
    plan.set_precision(P.PREC_FP32)
    b_fp32 = plan.run(delta_gpu).cpu().numpy()
    tri_all = plan.triangles.numpy()
    ntri_all = plan.ntri.numpy()
    plan.close()
    del delta_gpu
    index = {tuple(r): t for t, r in enumerate(tri_all.tolist())}
    sset = {1, 2, 64, 65, 127, 128}
    sample = [r for r in geometry.all_triangles(n_s).tolist() if set(r) <= sset]
    # and two triangles of every wavefront slot shape of the split-bf16 tiling,
    # preferring shells already sampled (each new shell is two 512^3 oracle fields)
    _, shape = P.bispec_contraction_tiles(P.make_config(n_g, box, dk, n_s, rsd_beta=beta)[0])
    shape = np.array(shape)
    chosen = {index[tuple(r)] for r in sample}
    for sh in np.unique(shape):
        cand = [t for t in np.nonzero(shape == sh)[0].tolist() if t not in chosen]
        for _ in range(2):
            if not cand:
                break
            t = max(cand, key=lambda q: (len(set(tri_all[q].tolist()) & sset), -q))
            cand.remove(t)
            chosen.add(t)
            sset |= set(tri_all[t].tolist())
    idx = np.array(sorted(chosen))
    sample = tri_all[idx].tolist()
    assert all(np.count_nonzero(shape[idx] == sh) >= min(2, np.count_nonzero(shape == sh)) for sh in np.unique(shape))
    say("sample: %d triangles over %d shells, %d slot shapes" % (len(idx), len(sset), len(np.unique(shape))))
    ref = fbe.estimate(delta64, box, dk, np.array(sample), rsd_beta=beta, with_abs=True)
    say("oracle %.1fs on %d triangles" % (time.time() - t0, len(sample)))
    assert np.array_equal(ntri_all[idx], ref["ntri"])
    for name, b in (("fp32", b_fp32), ("split-bf16", b_split)):
        m = metrics(b[idx], ref["B"], ref["S"])
        say(name, m)
        assert m["e_cond"] <= 1e-5 and m["e_norm"] <= 1e-5, (name, m)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("n_g", [640, 768])
def test_large_radix3_radix5_grids(n_g):
    """The forward transform at the large mixed-radix sizes (640 = 5 x 128,
    768 = 3 x 256; 16-column strided tiles in dynamic LDS), with 4 shells, so
    the shell passes and the contraction run on a small estimator grid: all
    closable triangles against the float64 oracle on the full grid.  The
    field is a seeded quadratic transform of white noise (non-zero B)."""
    import paper_2107_14564_amd as P
    box, dk, n_s = 2000.0, 1.0, 4
    g = np.random.default_rng(640 + n_g).standard_normal((n_g,) * 3).astype(np.float32)
    d32 = (g + np.float32(0.3) * (g * g - np.float32(1.0))).astype(np.float32)
    del g
    delta_gpu, delta64 = to_gpu(d32)
    del d32
    plan = P.Plan(n_g, box, dk, n_s, rsd_beta=0.5, precision=P.PREC_SPLITBF16)
    b = plan.run(delta_gpu).cpu().numpy()
    tri = plan.triangles.numpy()
    ntri = plan.ntri.numpy()
    say("n_g=%d G=%d n_tri=%d" % (n_g, plan.n_est, plan.n_tri))
    plan.close()
    del delta_gpu
    ref = fbe.estimate(delta64, box, dk, tri, rsd_beta=0.5, with_abs=True)
    assert np.array_equal(ntri, ref["ntri"])
    m = metrics(b, ref["B"], ref["S"])
    say("n_g=%d" % n_g, m)
    assert m["e_cond"] <= 1e-5 and m["e_norm"] <= 1e-5, m
