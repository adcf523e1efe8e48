"""Parity of the remaining workload configurations through the C ABI.

* The shape-grid workload: N_g = 256, L = 1000 Mpc, P = k^-1, f_NG = 1,
  40 shells of width 2 k_f, a1 in {2, 4, ..., 40} and a 20 x 20 (mu, t) grid
  (2398 triangles), in both contraction precisions, every triangle against
  the float64 oracle.
* The batched workload: the 64 heterogeneous realisations (N_g in
  {96, 128, 160}, 16-48 shells), run as one captured HIP graph; six members
  spanning the three grids and the largest and smallest shell counts are
  checked against the oracle on every triangle, from the second of two graph
  replays with eager work on the device between them.

Bar: N_tri exact, e_norm <= 1e-5 and max e_cond <= 1e-5."""
import time

import numpy as np
import pytest

from gpu_util import gpu_ok, metrics, say, to_gpu
from oracle import fbe
from synth import batch_field, batch_members, workload_field

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ok(), reason="needs a GPU")]

TOL = 1e-5


@pytest.mark.timeout(900)
def test_shape_grid_workload_all_triangles():
    import paper_2107_14564_amd as P
    t0 = time.time()
    dg, d64 = to_gpu(workload_field("ng256"))
    plan = P.Plan(256, 1000.0, 2.0, 40, tri_mode=P.TRI_MUT_GRID, k1_shells=list(range(2, 41, 2)), n_mu=20, n_t=20,
                  precision=P.PREC_FP32)
    assert plan.n_tri == 2398
    b32 = plan.run(dg).cpu().numpy()
    plan.set_precision(P.PREC_SPLITBF16)
    b16 = plan.run(dg).cpu().numpy()
    tri, ntri = plan.triangles.numpy(), plan.ntri.numpy()
    plan.close()
    say("gpu %.1fs" % (time.time() - t0))
    ref = fbe.estimate(d64, 1000.0, 2.0, tri, with_abs=True)
    say("oracle %.1fs" % (time.time() - t0))
    assert np.array_equal(ntri, ref["ntri"])
    for name, b in (("fp32", b32), ("split-bf16", b16)):
        m = metrics(b, ref["B"], ref["S"])
        say("  %s %s" % (name, m))
        assert m["e_norm"] <= TOL and m["e_cond"] <= TOL, (name, m)


CHECKED = [0, 17, 4, 40, 7, 29]   # (160, 48), (128, 42), (96, 31), (160, 17), (128, 16), (96, 19) shells


@pytest.mark.timeout(1100)
def test_batch_workload_members_in_graph_replay():
    import torch
    import paper_2107_14564_amd as P
    t0 = time.time()
    members = batch_members(64, 4999)
    fields = [np.ascontiguousarray(batch_field(m), dtype=np.float32) for m in members]
    configs = [dict(n_g=m["n_g"], box_l=m["box_l"], dk=1.0, n_shells=m["n_shells"]) for m in members]
    bp = P.BatchPlan(configs)
    say("batch plan %.1fs, %d triangles" % (time.time() - t0, bp.n_tri))
    packed = bp.pack([torch.from_numpy(f) for f in fields])
    out = torch.empty(bp.n_tri, dtype=torch.float64, device=packed.device)
    bp.run_into(packed, out, use_graph=True)
    torch.cuda.synchronize()
    first = out.clone()
    junk = torch.randn(1 << 20, device=packed.device) * 3.0   # eager work between the replays
    out.fill_(0.0)
    bp.run_into(packed, out, use_graph=True)
    torch.cuda.synchronize()
    del junk
    assert torch.equal(first, out), "graph replays differ"
    b = out.cpu().numpy()
    for i in CHECKED:
        m = members[i]
        tri = bp.triangles[i].numpy()
        ref = fbe.estimate(fields[i].astype(np.float64), m["box_l"], 1.0, tri, with_abs=True)
        assert np.array_equal(bp.ntri[i].numpy(), ref["ntri"]), "N_tri differs, member %d" % i
        mt = metrics(b[bp.b_off[i]:bp.b_off[i + 1]], ref["B"], ref["S"])
        say("  member %d n_g=%d n_s=%d n_tri=%d %s (%.0fs)" % (i, m["n_g"], m["n_shells"], len(tri), mt,
                                                               time.time() - t0))
        assert mt["e_norm"] <= TOL and mt["e_cond"] <= TOL, (i, mt)
    bp.close()
