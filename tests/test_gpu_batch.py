"""The batched form through the C ABI: heterogeneous members against the FP64
oracle, HIP-graph replays against direct launches, and autotuned plans.

Tolerances as in test_gpu_parity (e_norm and max e_cond <= 1e-5, N_tri exact);
graph replays must reproduce the directly launched batch bit for bit (the same
kernels in the same order)."""
import numpy as np
import pytest

from gpu_util import gpu_ok, metrics, say
from oracle import fbe
from synth import PowerLaw, gaussian_field, quadratic_ng_field

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ok(), reason="needs a GPU")]

TOL = 1e-5

# (n_g, box_l, dk, n_shells, rsd_beta, extra plan arguments)
MEMBERS = [
    (16, 100.0, 1.0, 4, 0.0, {}),
    (24, 60.0, 1.0, 6, 0.5, {"precision": 1}),
    (32, 300.0, 1.0, 10, 0.0, {"tri_mode": 2, "k1_shells": list(range(5, 11)), "n_mu": 10, "n_t": 10}),
    (40, 200.0, 1.0, 12, 0.5, {}),
    (48, 200.0, 1.5, 9, 1.0, {"tri_mode": 1, "k1_shells": [7, 9]}),
    (64, 300.0, 1.0, 8, 0.5, {}),            # estimator grid 32
]


def _configs():
    out = []
    for n_g, box, dk, n_s, beta, extra in MEMBERS:
        c = dict(n_g=n_g, box_l=box, dk=dk, n_shells=n_s, rsd_beta=beta)
        c.update(extra)
        out.append(c)
    return out


def _fields(seed0):
    return [quadratic_ng_field(gaussian_field(m[0], m[1], PowerLaw(-1.0), seed0 + i), 1.0).astype(np.float32)
            for i, m in enumerate(MEMBERS)]


def _check_members(bp, b, fields):
    for i, (m, d) in enumerate(zip(MEMBERS, fields)):
        n_g, box, dk, n_s, beta, _ = m
        tri = bp.triangles[i].numpy()
        ref = fbe.estimate(d.astype(np.float64), box, dk, tri, rsd_beta=beta, with_abs=True)
        assert np.array_equal(bp.ntri[i].numpy(), ref["ntri"]), "N_tri differs, member %d" % i
        got = b[bp.b_off[i]:bp.b_off[i + 1]]
        mt = metrics(got, ref["B"], ref["S"])
        say("  member %d n_g=%d n_tri=%d %s" % (i, n_g, len(tri), mt))
        assert mt["e_cond"] <= TOL and mt["e_norm"] <= TOL, (i, mt)


def test_batch_matches_oracle_eager_and_graph():
    import torch
    import paper_2107_14564_amd as P
    say("batch of %d members" % len(MEMBERS))
    bp = P.BatchPlan(_configs())
    fields = _fields(900)
    packed = bp.pack([torch.from_numpy(f) for f in fields])
    b_eager = bp.run(packed, use_graph=False).cpu().numpy()
    _check_members(bp, b_eager, fields)
    out = torch.empty(bp.n_tri, dtype=torch.float64, device=packed.device)
    # replays of one captured graph, with unrelated eager work and synchronisations between them
    x = torch.randn(512, 512, device=packed.device)
    for r in range(3):
        bp.run_into(packed, out, use_graph=True)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        say("  replay %d max |graph - eager| = %.3g" % (r, float(np.max(np.abs(got - b_eager)))))
        assert np.array_equal(got, b_eager), "graph replay %d differs from the direct launches" % r
        x = (x @ x.T) / 512.0
        out.zero_()
        torch.cuda.synchronize()
    # new inputs at a new address: the graph is captured again
    fields2 = _fields(950)
    packed2 = bp.pack([torch.from_numpy(f) for f in fields2])
    b2_graph = bp.run(packed2, use_graph=True).cpu().numpy()
    b2_eager = bp.run(packed2, use_graph=False).cpu().numpy()
    assert np.array_equal(b2_graph, b2_eager)
    _check_members(bp, b2_graph, fields2)
    bp.close()


def test_batch_members_match_single_plans():
    """A member of the batch computes exactly what the same plan alone computes."""
    import torch
    import paper_2107_14564_amd as P
    cfgs = _configs()
    bp = P.BatchPlan(cfgs)
    fields = _fields(700)
    b = bp.run(bp.pack([torch.from_numpy(f) for f in fields]), use_graph=True).cpu().numpy()
    for i, c in enumerate(cfgs):
        c = dict(c)
        plan = P.Plan(c.pop("n_g"), c.pop("box_l"), c.pop("dk"), c.pop("n_shells"), **c)
        single = plan.run(torch.from_numpy(fields[i]).cuda()).cpu().numpy()
        assert np.array_equal(single, b[bp.b_off[i]:bp.b_off[i + 1]]), i
        plan.close()
    bp.close()


def test_batch_cohorts():
    """Identical consecutive members form cohorts (one launch per pass for all of
    them, each member at its own strides): a batch A A A B A A C C (C a
    quadrupole plan) has the units (A A A), B, (A A), (C C); every member
    computes exactly what the same plan alone computes on its field, graph
    replays equal direct launches, and the last member of each A cohort
    matches the oracle."""
    import torch
    import paper_2107_14564_amd as P
    a = dict(n_g=48, box_l=200.0, dk=1.0, n_shells=12, rsd_beta=0.5)
    b = dict(n_g=32, box_l=300.0, dk=1.0, n_shells=10, rsd_beta=0.0)
    c = dict(n_g=32, box_l=300.0, dk=1.0, n_shells=8, rsd_beta=0.5, ell=2)
    cfgs = [a, a, a, b, a, a, c, c]
    bp = P.BatchPlan(cfgs)
    say("cohort batch: %d units, %d members in cohorts" % (bp.n_units, bp.n_cohort_members))
    assert (bp.n_units, bp.n_cohort_members) == (4, 7)
    fields = [quadratic_ng_field(gaussian_field(c["n_g"], c["box_l"], PowerLaw(-1.0), 300 + i), 1.0)
              .astype(np.float32) for i, c in enumerate(cfgs)]
    packed = bp.pack([torch.from_numpy(f) for f in fields])
    b_eager = bp.run(packed, use_graph=False).cpu().numpy()
    b_graph = bp.run(packed, use_graph=True).cpu().numpy()
    assert np.array_equal(b_graph, b_eager)
    for i, c in enumerate(cfgs):
        c = dict(c)
        plan = P.Plan(c.pop("n_g"), c.pop("box_l"), c.pop("dk"), c.pop("n_shells"), **c)
        single = plan.run(torch.from_numpy(fields[i]).cuda()).cpu().numpy()
        got = b_eager[bp.b_off[i]:bp.b_off[i + 1]]
        say("  member %d max |batch - single| = %.3g" % (i, float(np.max(np.abs(got - single)))))
        assert np.array_equal(single, got), i
        plan.close()
    for i in (2, 5):
        c = cfgs[i]
        ref = fbe.estimate(fields[i].astype(np.float64), c["box_l"], c["dk"], bp.triangles[i].numpy(),
                           rsd_beta=c["rsd_beta"], with_abs=True)
        mt = metrics(b_eager[bp.b_off[i]:bp.b_off[i + 1]], ref["B"], ref["S"])
        say("  member %d vs oracle %s" % (i, mt))
        assert np.array_equal(bp.ntri[i].numpy(), ref["ntri"])
        assert mt["e_cond"] <= TOL and mt["e_norm"] <= TOL
    bp.close()


def test_autotuned_plan(tmp_path, monkeypatch):
    """FLAG_AUTOTUNE picks each grid class's column-tile window and voxel-range
    count by timing; results stay within tolerance.  With BISPEC_TUNE_CACHE set,
    the choices are written to the cache, and a second plan of the same
    configuration reads them back (same choices, bit-identical B)."""
    import torch
    import paper_2107_14564_amd as P
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("BISPEC_TUNE_CACHE", str(cache))
    n_g, box = 64, 300.0
    d = quadratic_ng_field(gaussian_field(n_g, box, PowerLaw(-1.0), 71), 1.0).astype(np.float32)
    plan = P.Plan(n_g, box, 1.0, 20, rsd_beta=0.5, flags=P.FLAG_AUTOTUNE)
    tuned = plan.classes()
    say("autotuned classes %s" % tuned)
    assert all(c["tune_source"] == "timed" and c["tuned_ms"] > 0 and c["max_cols"] in (4, 8)
               and c["n_krange"] in (64, 128, 256, 512) for c in tuned)
    B = plan.run(torch.from_numpy(d).cuda()).cpu().numpy()
    ref = fbe.estimate(d.astype(np.float64), box, 1.0, plan.triangles.numpy(), rsd_beta=0.5, with_abs=True)
    mt = metrics(B, ref["B"], ref["S"])
    say("autotuned %s" % mt)
    assert np.array_equal(plan.ntri.numpy(), ref["ntri"])
    assert mt["e_cond"] <= TOL and mt["e_norm"] <= TOL
    assert len(cache.read_text().splitlines()) == len(tuned)
    plan2 = P.Plan(n_g, box, 1.0, 20, rsd_beta=0.5, flags=P.FLAG_AUTOTUNE)
    again = plan2.classes()
    assert [c["tune_source"] for c in again] == ["cache"] * len(tuned)
    assert [(c["max_cols"], c["n_krange"]) for c in again] == [(c["max_cols"], c["n_krange"]) for c in tuned]
    B2 = plan2.run(torch.from_numpy(d).cuda()).cpu().numpy()
    assert np.array_equal(B, B2)
    plan.close()
    plan2.close()


def test_batch_rejects_grad_flag():
    import paper_2107_14564_amd as P
    c = _configs()[:2]
    c[1]["flags"] = P.FLAG_GRAD
    with pytest.raises(P.BispecError) as e:
        P.BatchPlan(c)
    assert e.value.status == -1
