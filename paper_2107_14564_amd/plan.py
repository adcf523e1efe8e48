"""Plan objects and the autograd entry point (marshalling only)."""
from __future__ import annotations

import torch

from . import _abi


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


class Plan:
    """A bispectrum plan on the current device.

    Arguments follow bispec_config: grid size n_g, box side box_l, shell width
    dk (units of 2 pi / box_l), n_shells, optional RSD beta, a triangle
    selection (tri_mode with k1_shells / n_mu / n_t / triangles), the
    contraction precision, flags and the estimator grid n_est (0 = automatic:
    the smallest supported size above three times the largest mode component),
    order 4 for the fourth-order polyspectrum, and ell = 2 or 4 for a Legendre
    multipole of the redshift-space bispectrum (weight L_ell(mu) on the first
    side, line of sight z, times 2 ell + 1).
    """

    def __init__(self, n_g, box_l, dk, n_shells, rsd_beta=0.0, tri_mode=_abi.TRI_ALL, k1_shells=None, n_mu=0,
                 n_t=0, triangles=None, precision=_abi.PREC_SPLITBF16, flags=0, n_est=0, order=0, ell=0):
        if not torch.cuda.is_available():
            raise RuntimeError("Plan needs a HIP device")
        self.cfg, self._keep = _abi.make_config(n_g, box_l, dk, n_shells, rsd_beta, tri_mode, k1_shells, n_mu, n_t,
                                                triangles, precision, flags, n_est, order, ell)
        self.ell = int(ell)
        self.order = 4 if int(order) == 4 else 3
        self.n_g = int(n_g)
        self.n_est = _abi.bispec_estimator_grid(self.cfg)
        # estimator-grid classes: grids, shell ranges, class of each triangle
        self.class_grids, self.class_shell_lo, self.class_shell_hi, tc = _abi.bispec_grid_classes(self.cfg)
        self.tri_class = torch.tensor(tc, dtype=torch.int32)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.handle = _abi.bispec_plan(self.cfg, _stream())
        if self.order == 4:
            # bins of four shells; ntri holds N_quad
            abc, ntri = _abi.bispec_quads(self.handle)
            self.labels = torch.zeros((len(abc), 0), dtype=torch.float64)
        else:
            abc, lab, ntri = _abi.bispec_triangles(self.handle)
            self.labels = torch.tensor(lab, dtype=torch.float64)
        self.triangles = torch.tensor(abc, dtype=torch.int32)
        self.ntri = torch.tensor(ntri, dtype=torch.int64)
        self.n_tri = len(abc)
        # counts bispec_run calls: the plan's shell fields belong to the last run
        self.runs = 0
        # x-slabs per grid class (1: whole fields resident; more: streamed)
        self.slabs = _abi.bispec_plan_slabs(self.handle)

    def run(self, delta: torch.Tensor) -> torch.Tensor:
        self._check_field(delta)
        out = torch.empty(self.n_tri, dtype=torch.float64, device=delta.device)
        _abi.bispec_run(self.handle, delta.data_ptr(), out.data_ptr(), _stream())
        self.runs += 1
        return out

    def run_noalloc_into(self, delta: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """bispec_run_noalloc into a caller-allocated float64 [n_tri] tensor (the
        library allocates nothing; the run buffers live in its static scratch)."""
        self._check_field(delta)
        if out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous() or out.numel() != self.n_tri:
            raise ValueError("out must be a contiguous float64 CUDA tensor of n_tri elements")
        _abi.bispec_run_noalloc(self.handle, delta.data_ptr(), out.data_ptr(), _stream())
        return out

    def grad(self, g_b: torch.Tensor) -> torch.Tensor:
        g_b = g_b.to(dtype=torch.float64, device=self.device).contiguous()
        if g_b.numel() != self.n_tri:
            raise ValueError("gradient of B has the wrong length")
        out = torch.empty((self.n_g,) * 3, dtype=torch.float32, device=self.device)
        _abi.bispec_grad(self.handle, g_b.data_ptr(), out.data_ptr(), _stream())
        return out

    def set_precision(self, precision: int):
        _abi.bispec_set_precision(self.handle, precision)

    def stage_times(self):
        return _abi.bispec_stage_times(self.handle, 4)

    def field(self, shell: int) -> torch.Tensor:
        """Shell field D_n / (dV n_g^{3/2}) on the grid of field_grid(shell) (g^3 points)."""
        g = self.field_grid(shell)
        out = torch.empty((g,) * 3, dtype=torch.float32, device=self.device)
        _abi.bispec_copy_field(self.handle, shell, out.data_ptr(), _stream())
        return out

    def class_field(self, cls: int, shell: int) -> torch.Tensor:
        """Shell field of grid class cls (its grid class_grids[cls], g^3 points)."""
        g = self.class_grids[cls]
        out = torch.empty((g,) * 3, dtype=torch.float32, device=self.device)
        _abi.bispec_copy_class_field(self.handle, cls, shell, out.data_ptr(), _stream())
        return out

    def classes(self):
        """The grid classes as built: grid, voxel ranges, column-tile window,
        work groups, autotuned time and its source, per class."""
        return _abi.bispec_plan_classes(self.handle)

    def field_grid(self, shell: int) -> int:
        """The grid of the largest grid class whose fields cover this shell."""
        return _abi.bispec_field_grid(self.handle, shell)

    def _check_field(self, delta):
        if (delta.dtype != torch.float32 or not delta.is_cuda or not delta.is_contiguous()
                or tuple(delta.shape) != (self.n_g,) * 3):
            raise ValueError("delta must be a contiguous float32 CUDA tensor of shape (n_g, n_g, n_g)")

    def close(self):
        if getattr(self, "handle", None):
            _abi.bispec_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _BispecFn(torch.autograd.Function):
    """bispec_grad differentiates the plan's last run; when the plan has run on
    other fields since this forward, backward first runs it again on this
    forward's input (saved, so in-place changes to it raise), which restores
    the shell fields the vector-Jacobian product needs."""

    @staticmethod
    def forward(ctx, delta, plan):
        delta = delta.contiguous()
        ctx.plan = plan
        out = plan.run(delta)
        ctx.run_id = plan.runs
        ctx.save_for_backward(delta)
        return out

    @staticmethod
    def backward(ctx, g_b):
        (delta,) = ctx.saved_tensors
        plan = ctx.plan
        if plan.runs != ctx.run_id:
            plan.run(delta)
        return plan.grad(g_b), None


class BatchPlan:
    """Many configurations run back to back on one shared workspace (the batched
    form).  configs: a list of dicts with the Plan keyword arguments (n_g, box_l,
    dk, n_shells, rsd_beta, tri_mode, k1_shells, n_mu, n_t, triangles,
    precision, flags, n_est)."""

    def __init__(self, configs):
        if not torch.cuda.is_available():
            raise RuntimeError("BatchPlan needs a HIP device")
        self._keep = []
        cfgs = []
        for c in configs:
            c = dict(c)
            cfg, keep = _abi.make_config(c.pop("n_g"), c.pop("box_l"), c.pop("dk"), c.pop("n_shells"), **c)
            cfgs.append(cfg)
            self._keep.append(keep)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.handle = _abi.bispec_plan_many(cfgs, _stream())
        self.delta_off, self.b_off = _abi.bispec_many_layout(self.handle)
        self.n = len(cfgs)
        self.n_g = [int(round((self.delta_off[i + 1] - self.delta_off[i]) ** (1 / 3))) for i in range(self.n)]
        self.triangles, self.ntri = [], []
        for i in range(self.n):
            abc, _, ntri = _abi.bispec_triangles(_abi.bispec_many_plan(self.handle, i))
            self.triangles.append(torch.tensor(abc, dtype=torch.int32))
            self.ntri.append(torch.tensor(ntri, dtype=torch.int64))
        self.n_tri = self.b_off[-1]
        # launch units: cohorts of identical consecutive members and single members
        self.n_units, self.n_cohort_members = _abi.bispec_many_units(self.handle)

    def pack(self, deltas) -> torch.Tensor:
        """One contiguous float32 device buffer of the members' fields."""
        if len(deltas) != self.n:
            raise ValueError("one field per member")
        for d, n in zip(deltas, self.n_g):
            if tuple(d.shape) != (n,) * 3 or d.dtype != torch.float32:
                raise ValueError("member fields must be float32 (n_g, n_g, n_g)")
        return torch.cat([d.reshape(-1).to(self.device) for d in deltas])

    def run(self, packed: torch.Tensor, use_graph: bool = True) -> torch.Tensor:
        """Packed B (float64 [total n_tri]); split with self.split()."""
        if packed.dtype != torch.float32 or not packed.is_cuda or not packed.is_contiguous() \
                or packed.numel() != self.delta_off[-1]:
            raise ValueError("packed fields must be a contiguous float32 CUDA tensor of the batch's total size")
        out = torch.empty(self.n_tri, dtype=torch.float64, device=packed.device)
        _abi.bispec_run_many(self.handle, packed.data_ptr(), out.data_ptr(), use_graph, _stream())
        return out

    def run_into(self, packed: torch.Tensor, out: torch.Tensor, use_graph: bool = True) -> torch.Tensor:
        """As run, into a caller-kept output (a stable pointer keeps the captured graph)."""
        if out.dtype != torch.float64 or out.numel() != self.n_tri or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 tensor of the batch's total n_tri")
        _abi.bispec_run_many(self.handle, packed.data_ptr(), out.data_ptr(), use_graph, _stream())
        return out

    def classes(self, i: int):
        """Member i's grid classes as built (see Plan.classes)."""
        return _abi.bispec_plan_classes(_abi.bispec_many_plan(self.handle, i))

    def split(self, b: torch.Tensor):
        return [b[self.b_off[i]:self.b_off[i + 1]] for i in range(self.n)]

    def close(self):
        if getattr(self, "handle", None):
            _abi.bispec_destroy_many(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bispectrum(delta: torch.Tensor, plan: Plan) -> torch.Tensor:
    """B (float64 [n_tri]) of delta; differentiable when the plan has FLAG_GRAD."""
    return _BispecFn.apply(delta, plan)
