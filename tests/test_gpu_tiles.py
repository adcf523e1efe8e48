"""Every tile of the headline contraction against the float64 oracle.

N_g = 320 (L = 937.5 Mpc, the headline's cell size; P = k^-1.5, f_NG = 2,
RSD beta = 0.5, 100 shells of one k_f, all 89 625 closable triangles) is the
smallest grid that holds the headline's shells; its grid classes and their
split-bf16 tilings are those of the N_g = 512 headline plan (asserted on the
host tables), so this plan runs every tile and every wavefront slot shape
the benchmark runs.

* Oracle parity: from every 16 x 16 accumulator tile, the triangles with the
  smallest and largest a3 of one of its pairs (one or two per tile, over 1100
  in all), against the float64 oracle on the full 320^3 grid: N_tri exact,
  e_norm and max e_cond <= 1e-5, in both contraction precisions.
* Every triangle, per triangle: the split-bf16 and fp32 results against a
  float64 contraction (torch, on the device) of the plan's own shell fields,
  read back per grid class, and against each other, within 1e-5 of the
  triangle's summation scale S_t = sum_x |F_a1 F_a2 F_a3| (same normalisation
  as B).  This isolates the contraction's arithmetic and tile maps on all
  89 625 triangles; the oracle comparison above covers the fields."""
import time

import numpy as np
import pytest

from gpu_util import gpu_ok, metrics, say, to_gpu
from oracle import fbe
from synth import workload_field

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ok(), reason="needs a GPU")]

N_G, BOX, DK, N_S, BETA = 320, 937.5, 1.0, 100, 0.5
TOL = 1e-5


@pytest.fixture(scope="module")
def headline_tiles():
    import torch
    import paper_2107_14564_amd as P
    t0 = time.time()
    cfg = P.make_config(N_G, BOX, DK, N_S, rsd_beta=BETA)[0]
    tile, shape = (np.array(v) for v in P.bispec_contraction_tiles(cfg))
    t512, s512 = (np.array(v) for v in P.bispec_contraction_tiles(P.make_config(512, 1500.0, DK, N_S,
                                                                                 rsd_beta=BETA)[0]))
    assert np.array_equal(tile, t512) and np.array_equal(shape, s512), "tiling differs from the headline plan"
    dg, d64 = to_gpu(workload_field("ng320"))
    plan = P.Plan(N_G, BOX, DK, N_S, rsd_beta=BETA, precision=P.PREC_SPLITBF16)
    assert plan.n_tri == 89625
    b16 = plan.run(dg).cpu().numpy()
    plan.set_precision(P.PREC_FP32)
    b32 = plan.run(dg).cpu().numpy()
    tri, ntri = plan.triangles.numpy(), plan.ntri.numpy()
    say("gpu %.1fs: %d tiles, %d slot shapes, classes %s" % (time.time() - t0, len(set(tile.tolist())),
                                                             len(set(shape.tolist())), plan.class_grids))
    # float64 contraction of the plan's own fields, class by class, and the summation scale
    vol = BOX ** 3
    dv = vol / N_G ** 3
    b64 = np.zeros(plan.n_tri)
    s_b = np.zeros(plan.n_tri)
    tc = plan.tri_class.numpy()
    for k, (g, lo, hi) in enumerate(zip(plan.class_grids, plan.class_shell_lo, plan.class_shell_hi)):
        F = torch.stack([plan.class_field(k, n).double().reshape(-1) for n in range(lo, hi + 1)])
        A = F.abs()
        idx = np.nonzero(tc == k)[0]
        pairs = {}
        for t in idx:
            pairs.setdefault((int(tri[t, 0]), int(tri[t, 1])), []).append(t)
        for (a1, a2), ts in pairs.items():
            rows = torch.tensor([int(tri[t, 2]) - lo for t in ts], device=F.device)
            T = (F.index_select(0, rows) @ (F[a1 - lo] * F[a2 - lo])).cpu().numpy()
            S = (A.index_select(0, rows) @ (A[a1 - lo] * A[a2 - lo])).cpu().numpy()
            norm = (dv * N_G ** 1.5) ** 3 / (vol * ntri[ts].astype(np.float64) * float(g) ** 3)
            b64[ts] = T * norm
            s_b[ts] = S * norm
        del F, A
        torch.cuda.empty_cache()
    say("float64 contraction of the plan's fields %.1fs" % (time.time() - t0))
    plan.close()
    return dict(tri=tri, ntri=ntri, b16=b16, b32=b32, b64=b64, s_b=s_b, tile=tile, shape=shape, d64=d64)


def test_every_triangle_against_a_float64_contraction_of_the_same_fields(headline_tiles):
    h = headline_tiles
    for name, b in (("split-bf16", h["b16"]), ("fp32", h["b32"])):
        e = np.abs(b - h["b64"]) / h["s_b"]
        worst = int(np.argmax(e))
        say("  %s vs float64 contraction: max e_cond %.3g at %s (shape %d)" % (name, e[worst], h["tri"][worst],
                                                                             h["shape"][worst]))
        assert np.all(e <= TOL), (name, e[worst])
    e = np.abs(h["b16"] - h["b32"]) / h["s_b"]
    say("  split-bf16 vs fp32 per triangle: max %.3g" % e.max())
    assert np.all(e <= TOL)


def test_every_tile_against_the_oracle(headline_tiles):
    h = headline_tiles
    tri, tile = h["tri"], h["tile"]
    sample = []
    for tl in np.unique(tile):
        ts = np.nonzero(tile == tl)[0]
        by_pair = {}
        for t in ts:
            by_pair.setdefault((int(tri[t, 0]), int(tri[t, 1])), []).append(t)
        ts = max(by_pair.values(), key=len)
        a3 = tri[ts, 2]
        sample += sorted({ts[int(np.argmin(a3))], ts[int(np.argmax(a3))]})
    sample = np.array(sorted(sample))
    shapes = h["shape"][sample]
    assert len(np.unique(tile[sample])) == len(np.unique(tile))
    assert all(np.count_nonzero(shapes == s) >= 2 for s in np.unique(h["shape"]))
    t0 = time.time()
    ref = fbe.estimate(h["d64"], BOX, DK, tri[sample], rsd_beta=BETA, with_abs=True)
    say("oracle %.1fs on %d triangles from %d tiles" % (time.time() - t0, len(sample), len(np.unique(tile))))
    assert np.array_equal(h["ntri"][sample], ref["ntri"])
    for name, b in (("split-bf16", h["b16"]), ("fp32", h["b32"])):
        m = metrics(b[sample], ref["B"], ref["S"])
        say("  %s %s" % (name, m))
        for s in np.unique(shapes):
            k = shapes == s
            e = float(np.max(np.abs(b[sample][k] - ref["B"][k]) / ref["S"][k]))
            assert e <= TOL, (name, "shape", s // 16, s % 16, e)
        assert m["e_norm"] <= TOL and m["e_cond"] <= TOL, (name, m)
