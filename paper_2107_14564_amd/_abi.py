"""ctypes binding of libbispec.so (include/bispec.h): argument marshalling only.

Every function here has the name of the C entry point it calls.  All arithmetic
runs in the HIP library; if the library is missing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbispec.so")

BISPEC_OK, BISPEC_EINVAL, BISPEC_ECUTOFF, BISPEC_ENOMEM = 0, -1, -2, -3
BISPEC_EHIP, BISPEC_ESTATE, BISPEC_EPREC = -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ECUTOFF", -3: "ENOMEM", -4: "EHIP", -5: "ESTATE", -6: "EPREC"}
TRI_ALL, TRI_K1SET, TRI_MUT_GRID, TRI_LIST = 0, 1, 2, 3
PREC_SPLITBF16, PREC_FP32 = 0, 1
FLAG_GRAD, FLAG_STAGE_TIMING, FLAG_AUTOTUNE, FLAG_NO_WORKSPACE, FLAG_ONE_GRID = 1, 2, 4, 8, 16


class BispecError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__("%s failed with %s: %s" % (where, STATUS_NAMES.get(status, status), message))
        self.status = status


class bispec_config(C.Structure):
    _fields_ = [
        ("n_g", C.c_int32), ("n_shells", C.c_int32), ("box_l", C.c_double), ("dk", C.c_double),
        ("rsd_beta", C.c_double), ("tri_mode", C.c_int32), ("n_k1", C.c_int32),
        ("k1_shells", C.POINTER(C.c_int32)), ("n_mu", C.c_int32), ("n_t", C.c_int32),
        ("n_list", C.c_int64), ("list", C.POINTER(C.c_int32)), ("precision", C.c_int32),
        ("flags", C.c_uint32), ("n_est", C.c_int32), ("order", C.c_int32), ("ell", C.c_int32),
    ]


_lib = None


def lib() -> C.CDLL:
    """The loaded HIP library; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libbispec.so is not built (run __graft_entry__.build() or "
                               "python -m paper_2107_14564_amd.build)")
        L = C.CDLL(LIB_PATH)
        P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        cfgp = C.POINTER(bispec_config)
        sig = {
            "bispec_query_triangles": [cfgp, C.POINTER(I64), C.POINTER(I32), C.POINTER(D), I64],
            "bispec_shell_stats": [cfgp, C.POINTER(I64), C.POINTER(D)],
            "bispec_workspace_bytes": [cfgp, C.POINTER(I64), C.POINTER(I64)],
            "bispec_estimator_grid": [cfgp, C.POINTER(I32)],
            "bispec_grid_classes": [cfgp, C.POINTER(I32), C.POINTER(I32), C.POINTER(I32), C.POINTER(I32), I32,
                                    C.POINTER(I32)],
            "bispec_field_grid": [P, I32, C.POINTER(I32)],
            "bispec_contraction_tiles": [cfgp, I64, C.POINTER(I32), C.POINTER(I32)],
            "bispec_copy_class_field": [P, I32, I32, P, P],
            "bispec_query_quads": [cfgp, C.POINTER(I64), C.POINTER(I32), I64],
            "bispec_quads": [P, C.POINTER(I32), C.POINTER(I64)],
            "bispec_plan_classes": [P, I32, C.POINTER(I32), C.POINTER(I32), C.POINTER(I32), C.POINTER(I32),
                                    C.POINTER(I32), C.POINTER(I32), C.POINTER(C.c_float), C.POINTER(I32)],
            "bispec_plan": [cfgp, P, C.POINTER(P)],
            "bispec_plan_slabs": [P, C.POINTER(I32)],
            "bispec_num_triangles": [P, C.POINTER(I64)],
            "bispec_triangles": [P, C.POINTER(I32), C.POINTER(D), C.POINTER(I64)],
            "bispec_run": [P, P, P, P],
            "bispec_run_noalloc": [P, P, P, P],
            "bispec_grad": [P, P, P, P],
            "bispec_set_precision": [P, I32],
            "bispec_stage_times": [P, C.POINTER(C.c_float), I32],
            "bispec_copy_field": [P, I32, P, P],
            "bispec_destroy": [P],
            "bispec_plan_many": [cfgp, I32, P, C.POINTER(P)],
            "bispec_many_layout": [P, C.POINTER(I32), C.POINTER(I64), C.POINTER(I64)],
            "bispec_many_plan": [P, I32, C.POINTER(P)],
            "bispec_many_units": [P, C.POINTER(I32), C.POINTER(I32)],
            "bispec_run_many": [P, P, P, I32, P],
            "bispec_destroy_many": [P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.bispec_last_error.argtypes = []
        L.bispec_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(status: int, where: str):
    if status != BISPEC_OK:
        raise BispecError(status, where, lib().bispec_last_error().decode())


def _i32_array(values):
    if values is None:
        return None, 0
    vals = [int(v) for v in values]
    arr = (C.c_int32 * max(1, len(vals)))(*vals)
    return arr, len(vals)


def make_config(n_g, box_l, dk, n_shells, rsd_beta=0.0, tri_mode=TRI_ALL, k1_shells=None, n_mu=0, n_t=0,
                triangles=None, precision=PREC_SPLITBF16, flags=0, n_est=0, order=0, ell=0):
    """A bispec_config plus the ctypes arrays it points into (keep both alive)."""
    k1, nk1 = _i32_array(k1_shells)
    flat = None if triangles is None else [int(v) for row in triangles for v in row]
    lst, nflat = _i32_array(flat)
    width = 4 if int(order) == 4 else 3
    cfg = bispec_config(n_g=int(n_g), n_shells=int(n_shells), box_l=float(box_l), dk=float(dk),
                        rsd_beta=float(rsd_beta), tri_mode=int(tri_mode), n_k1=nk1,
                        k1_shells=C.cast(k1, C.POINTER(C.c_int32)) if k1 is not None else None,
                        n_mu=int(n_mu), n_t=int(n_t), n_list=nflat // width,
                        list=C.cast(lst, C.POINTER(C.c_int32)) if lst is not None else None,
                        precision=int(precision), flags=int(flags), n_est=int(n_est), order=int(order),
                        ell=int(ell))
    return cfg, (k1, lst)


def bispec_query_triangles(cfg):
    """(abc int32 [n][3], k1_mu_t float64 [n][3]) as Python lists of tuples."""
    n = C.c_int64(0)
    _check(lib().bispec_query_triangles(C.byref(cfg), C.byref(n), None, None, 0), "bispec_query_triangles")
    abc = (C.c_int32 * (3 * n.value))()
    lab = (C.c_double * (3 * n.value))()
    _check(lib().bispec_query_triangles(C.byref(cfg), C.byref(n), abc, lab, n.value), "bispec_query_triangles")
    return ([tuple(abc[3 * t:3 * t + 3]) for t in range(n.value)],
            [tuple(lab[3 * t:3 * t + 3]) for t in range(n.value)])


def bispec_shell_stats(cfg):
    ns = cfg.n_shells
    counts = (C.c_int64 * ns)()
    means = (C.c_double * ns)()
    _check(lib().bispec_shell_stats(C.byref(cfg), counts, means), "bispec_shell_stats")
    return list(counts), list(means)


def bispec_workspace_bytes(cfg):
    run, peak = C.c_int64(0), C.c_int64(0)
    _check(lib().bispec_workspace_bytes(C.byref(cfg), C.byref(run), C.byref(peak)), "bispec_workspace_bytes")
    return run.value, peak.value


def bispec_estimator_grid(cfg) -> int:
    n = C.c_int32(0)
    _check(lib().bispec_estimator_grid(C.byref(cfg), C.byref(n)), "bispec_estimator_grid")
    return n.value


def bispec_grid_classes(cfg):
    """(grids, shell_lo, shell_hi, tri_class): the plan's estimator-grid classes
    (grids ascending, inclusive 1-based shell ranges) and each triangle's class."""
    n = C.c_int32(0)
    _check(lib().bispec_grid_classes(C.byref(cfg), C.byref(n), None, None, None, 0, None), "bispec_grid_classes")
    k = n.value
    grid, lo, hi = (C.c_int32 * k)(), (C.c_int32 * k)(), (C.c_int32 * k)()
    n_tri = C.c_int64(0)
    if cfg.order == 4:
        _check(lib().bispec_query_quads(C.byref(cfg), C.byref(n_tri), None, 0), "bispec_query_quads")
    else:
        _check(lib().bispec_query_triangles(C.byref(cfg), C.byref(n_tri), None, None, 0), "bispec_query_triangles")
    tc = (C.c_int32 * max(1, n_tri.value))()
    _check(lib().bispec_grid_classes(C.byref(cfg), C.byref(n), grid, lo, hi, k, tc), "bispec_grid_classes")
    return list(grid), list(lo), list(hi), list(tc)[:n_tri.value]


def bispec_contraction_tiles(cfg):
    """(tile, shape) per selected triangle: its split-bf16 accumulator tile (unique
    over the plan) and the 16 NT + NRB shape of the wavefront slot owning it."""
    n_tri = C.c_int64(0)
    _check(lib().bispec_query_triangles(C.byref(cfg), C.byref(n_tri), None, None, 0), "bispec_query_triangles")
    n = n_tri.value
    tile, shape = (C.c_int32 * max(1, n))(), (C.c_int32 * max(1, n))()
    _check(lib().bispec_contraction_tiles(C.byref(cfg), n, tile, shape), "bispec_contraction_tiles")
    return list(tile)[:n], list(shape)[:n]


def bispec_plan_classes(plan: int):
    """Per grid class of a built plan: dict(grid, n_krange, max_cols, n_wg, tuned_ms, tune_source)."""
    n = C.c_int32(0)
    _check(lib().bispec_plan_classes(C.c_void_p(plan), 0, C.byref(n), None, None, None, None, None, None, None),
           "bispec_plan_classes")
    k = n.value
    g, kr, mc, wg, rp, src = ((C.c_int32 * max(1, k))() for _ in range(6))
    ms = (C.c_float * max(1, k))()
    _check(lib().bispec_plan_classes(C.c_void_p(plan), k, C.byref(n), g, kr, mc, wg, rp, ms, src),
           "bispec_plan_classes")
    return [dict(grid=g[i], n_krange=kr[i], max_cols=mc[i], n_wg=wg[i], rep=rp[i], tuned_ms=float(ms[i]),
                 tune_source=("default", "timed", "cache")[src[i]]) for i in range(k)]


def bispec_plan_slabs(plan: int) -> int:
    """x-slabs per grid class of a built plan (1: whole fields resident)."""
    n = C.c_int32(0)
    _check(lib().bispec_plan_slabs(C.c_void_p(plan), C.byref(n)), "bispec_plan_slabs")
    return n.value


def bispec_query_quads(cfg):
    """Selected quadruples (a1, a2, a3, a4) of an order-4 configuration."""
    n = C.c_int64(0)
    _check(lib().bispec_query_quads(C.byref(cfg), C.byref(n), None, 0), "bispec_query_quads")
    q = (C.c_int32 * max(1, 4 * n.value))()
    _check(lib().bispec_query_quads(C.byref(cfg), C.byref(n), q, n.value), "bispec_query_quads")
    return [tuple(q[4 * t:4 * t + 4]) for t in range(n.value)]


def bispec_quads(plan: int):
    """(abcd, nquad) of an order-4 plan."""
    n = C.c_int64(0)
    _check(lib().bispec_num_triangles(C.c_void_p(plan), C.byref(n)), "bispec_num_triangles")
    q = (C.c_int32 * max(1, 4 * n.value))()
    nq = (C.c_int64 * max(1, n.value))()
    _check(lib().bispec_quads(C.c_void_p(plan), q, nq), "bispec_quads")
    return [tuple(q[4 * t:4 * t + 4]) for t in range(n.value)], list(nq)[:n.value]


def bispec_field_grid(plan: int, shell: int) -> int:
    g = C.c_int32(0)
    _check(lib().bispec_field_grid(C.c_void_p(plan), int(shell), C.byref(g)), "bispec_field_grid")
    return g.value


def bispec_plan(cfg, stream: int = 0) -> int:
    h = C.c_void_p()
    _check(lib().bispec_plan(C.byref(cfg), C.c_void_p(stream), C.byref(h)), "bispec_plan")
    return h.value


def bispec_num_triangles(plan: int) -> int:
    n = C.c_int64(0)
    _check(lib().bispec_num_triangles(C.c_void_p(plan), C.byref(n)), "bispec_num_triangles")
    return n.value


def bispec_triangles(plan: int):
    n = bispec_num_triangles(plan)
    abc = (C.c_int32 * (3 * n))()
    lab = (C.c_double * (3 * n))()
    ntri = (C.c_int64 * n)()
    _check(lib().bispec_triangles(C.c_void_p(plan), abc, lab, ntri), "bispec_triangles")
    return ([tuple(abc[3 * t:3 * t + 3]) for t in range(n)],
            [tuple(lab[3 * t:3 * t + 3]) for t in range(n)], list(ntri))


def bispec_run(plan: int, delta_ptr: int, b_ptr: int, stream: int = 0):
    _check(lib().bispec_run(C.c_void_p(plan), C.c_void_p(delta_ptr), C.c_void_p(b_ptr), C.c_void_p(stream)),
           "bispec_run")


def bispec_run_noalloc(plan: int, delta_ptr: int, b_ptr: int, stream: int = 0):
    _check(lib().bispec_run_noalloc(C.c_void_p(plan), C.c_void_p(delta_ptr), C.c_void_p(b_ptr),
                                    C.c_void_p(stream)), "bispec_run_noalloc")


def bispec_grad(plan: int, gb_ptr: int, gdelta_ptr: int, stream: int = 0):
    _check(lib().bispec_grad(C.c_void_p(plan), C.c_void_p(gb_ptr), C.c_void_p(gdelta_ptr), C.c_void_p(stream)),
           "bispec_grad")


def bispec_set_precision(plan: int, precision: int):
    _check(lib().bispec_set_precision(C.c_void_p(plan), int(precision)), "bispec_set_precision")


def bispec_stage_times(plan: int, n: int = 4):
    ms = (C.c_float * n)()
    _check(lib().bispec_stage_times(C.c_void_p(plan), ms, n), "bispec_stage_times")
    return list(ms)


def bispec_copy_field(plan: int, shell: int, dst_ptr: int, stream: int = 0):
    _check(lib().bispec_copy_field(C.c_void_p(plan), int(shell), C.c_void_p(dst_ptr), C.c_void_p(stream)),
           "bispec_copy_field")


def bispec_copy_class_field(plan: int, cls: int, shell: int, dst_ptr: int, stream: int = 0):
    _check(lib().bispec_copy_class_field(C.c_void_p(plan), int(cls), int(shell), C.c_void_p(dst_ptr),
                                         C.c_void_p(stream)), "bispec_copy_class_field")


def bispec_destroy(plan: int):
    _check(lib().bispec_destroy(C.c_void_p(plan)), "bispec_destroy")


def bispec_plan_many(cfgs, stream: int = 0) -> int:
    """cfgs: a list of bispec_config structures (copied into one array)."""
    arr = (bispec_config * len(cfgs))(*cfgs)
    h = C.c_void_p()
    _check(lib().bispec_plan_many(arr, len(cfgs), C.c_void_p(stream), C.byref(h)), "bispec_plan_many")
    return h.value


def bispec_many_layout(batch: int):
    n = C.c_int32(0)
    _check(lib().bispec_many_layout(C.c_void_p(batch), C.byref(n), None, None), "bispec_many_layout")
    d = (C.c_int64 * (n.value + 1))()
    b = (C.c_int64 * (n.value + 1))()
    _check(lib().bispec_many_layout(C.c_void_p(batch), None, d, b), "bispec_many_layout")
    return list(d), list(b)


def bispec_many_units(batch: int):
    """(launch units, members in cohorts) of a batch."""
    u, c = C.c_int32(0), C.c_int32(0)
    _check(lib().bispec_many_units(C.c_void_p(batch), C.byref(u), C.byref(c)), "bispec_many_units")
    return u.value, c.value


def bispec_many_plan(batch: int, i: int) -> int:
    h = C.c_void_p()
    _check(lib().bispec_many_plan(C.c_void_p(batch), int(i), C.byref(h)), "bispec_many_plan")
    return h.value


def bispec_run_many(batch: int, delta_ptr: int, b_ptr: int, use_graph: bool = True, stream: int = 0):
    _check(lib().bispec_run_many(C.c_void_p(batch), C.c_void_p(delta_ptr), C.c_void_p(b_ptr), int(bool(use_graph)),
                                 C.c_void_p(stream)), "bispec_run_many")


def bispec_destroy_many(batch: int):
    _check(lib().bispec_destroy_many(C.c_void_p(batch)), "bispec_destroy_many")


def bispec_last_error() -> str:
    return lib().bispec_last_error().decode()
