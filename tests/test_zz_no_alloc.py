"""bispec_run_noalloc (the entry point for callers that cannot allocate)
against bispec_run on the same configuration, through the C ABI: two calls
in a row on one device, the second with a smaller grid and plan (so it runs
in scratch the first call left dirty), both split-bf16 and fp32.  The two
entry points run the same kernels in the same order, so B must agree bit for
bit; N_tri is the plan's in both.  Also: a plan made with
BISPEC_FLAG_NO_WORKSPACE refuses bispec_run (ESTATE), and a plan whose run
buffers exceed the static scratch is refused (EINVAL) before any launch."""
import numpy as np
import pytest

from gpu_util import gpu_ok, say
from synth import PowerLaw, gaussian_field, quadratic_ng_field

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ok(), reason="needs a GPU")]

# (n_g, box, n_shells, beta, precision): the larger first, then a smaller one
CASES = [(64, 300.0, 20, 0.0, 0), (32, 300.0, 10, 0.5, 1)]


def _field(n_g, box, seed):
    d = quadratic_ng_field(gaussian_field(n_g, box, PowerLaw(-1.0), seed), 1.0)
    return np.ascontiguousarray(d, dtype=np.float32)


def test_noalloc_matches_run_two_calls():
    import torch
    import paper_2107_14564_amd as P
    for k, (n_g, box, n_s, beta, prec) in enumerate(CASES):
        say("noalloc call %d: n_g=%d n_s=%d beta=%g precision=%d" % (k, n_g, n_s, beta, prec))
        d = torch.from_numpy(_field(n_g, box, 610 + k)).cuda()
        ref_plan = P.Plan(n_g, box, 1.0, n_s, rsd_beta=beta, precision=prec)
        na_plan = P.Plan(n_g, box, 1.0, n_s, rsd_beta=beta, precision=prec, flags=P.FLAG_NO_WORKSPACE)
        assert torch.equal(ref_plan.ntri, na_plan.ntri)
        b_ref = ref_plan.run(d)
        b_na = torch.full_like(b_ref, float("nan"))
        na_plan.run_noalloc_into(d, b_na)
        torch.cuda.synchronize()
        say("  n_tri=%d max|diff|=%g" % (ref_plan.n_tri, float((b_ref - b_na).abs().max())))
        assert torch.equal(b_ref, b_na)
        # the plan with its own workspace may use the scratch as well
        b_na2 = torch.full_like(b_ref, float("nan"))
        ref_plan.run_noalloc_into(d, b_na2)
        torch.cuda.synchronize()
        assert torch.equal(b_ref, b_na2)
        with pytest.raises(P.BispecError) as e:
            na_plan.run(d)
        assert e.value.status == -5
        ref_plan.close()
        na_plan.close()


def test_noalloc_refuses_plans_beyond_the_scratch():
    import torch
    import paper_2107_14564_amd as P
    plan = P.Plan(96, 300.0, 1.0, 31, flags=P.FLAG_NO_WORKSPACE)
    d = torch.zeros((96,) * 3, dtype=torch.float32, device="cuda")
    out = torch.empty(plan.n_tri, dtype=torch.float64, device="cuda")
    with pytest.raises(P.BispecError) as e:
        plan.run_noalloc_into(d, out)
    assert e.value.status == -1 and "scratch" in str(e.value)
    plan.close()
