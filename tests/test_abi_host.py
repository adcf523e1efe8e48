"""The C ABI on the host (no GPU): symbols, configuration checks, shell
geometry and triangle selection against the oracle's independent enumeration."""
import math
import os
import re

import numpy as np
import pytest

from oracle import geometry

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
abi = pytest.importorskip("paper_2107_14564_amd._abi")


def _header_symbols():
    txt = open(os.path.join(ROOT, "include", "bispec.h")).read()
    return set(re.findall(r"^\s*(?:int|const char\*)\s+(bispec_\w+)\s*\(", txt, re.M))


def test_library_exports_every_declared_symbol():
    L = abi.lib()
    syms = _header_symbols()
    assert len(syms) >= 13
    for s in syms:
        assert hasattr(L, s), s


def test_errors_are_reported():
    with pytest.raises(abi.BispecError) as e:
        abi.bispec_query_triangles(abi.make_config(32, 300.0, 1.0, 11)[0])
    assert e.value.status == abi.BISPEC_ECUTOFF
    for bad in [dict(n_g=33), dict(n_g=4), dict(n_g=14), dict(dk=0.5), dict(box_l=-1.0), dict(n_shells=0)]:
        kw = dict(n_g=32, box_l=300.0, dk=1.0, n_shells=4)
        kw.update(bad)
        with pytest.raises(abi.BispecError) as e:
            abi.bispec_query_triangles(abi.make_config(**kw)[0])
        assert e.value.status == abi.BISPEC_EINVAL, bad
    with pytest.raises(abi.BispecError):
        abi.bispec_query_triangles(abi.make_config(32, 300.0, 1.0, 4, tri_mode=abi.TRI_LIST,
                                                   triangles=[(3, 1, 1)])[0])   # not closable
    with pytest.raises(abi.BispecError):
        abi.bispec_query_triangles(abi.make_config(32, 300.0, 1.0, 4, tri_mode=abi.TRI_LIST,
                                                   triangles=[(2, 1, 1), (2, 1, 1)])[0])
    assert "closable" in abi.bispec_last_error() or "duplicate" in abi.bispec_last_error()
    # empty selections are rejected at plan time (a plan always has >= 1 triangle)
    for kw in [dict(tri_mode=abi.TRI_LIST, triangles=[]), dict(tri_mode=abi.TRI_K1SET, k1_shells=[]),
               dict(tri_mode=abi.TRI_MUT_GRID, k1_shells=[3], n_mu=0, n_t=5),
               dict(tri_mode=abi.TRI_K1SET, k1_shells=[9])]:
        with pytest.raises(abi.BispecError) as e:
            abi.bispec_query_triangles(abi.make_config(32, 300.0, 1.0, 4, **kw)[0])
        assert e.value.status == abi.BISPEC_EINVAL, kw
        assert abi.bispec_last_error(), kw


def test_cutoff_boundary():
    # (n_s + 1/2) w <= N/3: N = 24, w = 1 allows 7 shells, not 8; w = 2 allows 3
    abi.bispec_query_triangles(abi.make_config(24, 50.0, 1.0, 7)[0])
    abi.bispec_query_triangles(abi.make_config(24, 50.0, 2.0, 3)[0])
    for ns, w in [(8, 1.0), (4, 2.0)]:
        with pytest.raises(abi.BispecError):
            abi.bispec_query_triangles(abi.make_config(24, 50.0, w, ns)[0])


@pytest.mark.parametrize("w,ns", [(1.0, 10), (2.0, 15), (1.5, 12), (1.0, 100)])
def test_shell_stats_match_oracle(w, ns):
    cfg, _ = abi.make_config(1024, 1000.0, w, ns)
    counts, means = abi.bispec_shell_stats(cfg)
    oc, om = geometry.shell_stats(w, ns)
    assert list(oc) == counts
    kf = 2 * math.pi / 1000.0
    np.testing.assert_allclose(np.array(means), kf * om, rtol=1e-12)


@pytest.mark.parametrize("mode", ["all", "k1set", "grid_c1", "grid_c2", "list"])
def test_triangle_selection_matches_oracle(mode):
    L = 300.0
    if mode == "all":
        cfg, _ = abi.make_config(64, L, 1.0, 20)
        ref = geometry.all_triangles(20)
    elif mode == "k1set":
        cfg, _ = abi.make_config(64, L, 1.0, 20, tri_mode=abi.TRI_K1SET, k1_shells=[20, 7, 13])
        ref = geometry.all_triangles(20, k1_set=[7, 13, 20])
    elif mode == "grid_c1":
        cfg, _ = abi.make_config(32, L, 1.0, 10, tri_mode=abi.TRI_MUT_GRID, k1_shells=range(5, 11), n_mu=10, n_t=10)
        ref, _ = geometry.grid_triangles(range(5, 11), 10, 10)
    elif mode == "grid_c2":
        cfg, _ = abi.make_config(256, 1000.0, 2.0, 40, tri_mode=abi.TRI_MUT_GRID, k1_shells=range(2, 41, 2),
                                 n_mu=20, n_t=20)
        ref, _ = geometry.grid_triangles(range(2, 41, 2), 20, 20)
    else:
        rows = [(9, 5, 4), (3, 2, 2), (9, 9, 1), (5, 3, 3)]
        cfg, _ = abi.make_config(32, L, 1.0, 10, tri_mode=abi.TRI_LIST, triangles=rows)
        ref = np.array(sorted(rows))
    abc, lab = abi.bispec_query_triangles(cfg)
    assert [tuple(r) for r in np.asarray(ref).tolist()] == abc
    w = cfg.dk
    _, om = geometry.shell_stats(w, cfg.n_shells)
    k1, mu, t = geometry.labels(np.array(abc), om * 2 * math.pi / cfg.box_l)
    np.testing.assert_allclose(np.array(lab), np.stack([k1, mu, t], 1), rtol=1e-12)


def test_known_counts():
    """Closable-triple counts for the named workloads: 125 (N_g=32 shape grid), 2398
    (N_g=256 shape grid), 89625 (100 shells), 494 (30 shells, a1 in {29, 30})."""
    c1 = abi.make_config(32, 300.0, 1.0, 10, tri_mode=abi.TRI_MUT_GRID, k1_shells=range(5, 11), n_mu=10, n_t=10)[0]
    c2 = abi.make_config(256, 1000.0, 2.0, 40, tri_mode=abi.TRI_MUT_GRID, k1_shells=range(2, 41, 2), n_mu=20,
                         n_t=20)[0]
    c3 = abi.make_config(512, 1500.0, 1.0, 100, rsd_beta=0.5)[0]
    c5 = abi.make_config(256, 1000.0, 1.0, 30, tri_mode=abi.TRI_K1SET, k1_shells=[29, 30])[0]
    assert [len(abi.bispec_query_triangles(c)[0]) for c in (c1, c2, c3, c5)] == [125, 2398, 89625, 494]


def test_workspace_bytes():
    cfg = abi.make_config(512, 1500.0, 1.0, 100, rsd_beta=0.5)[0]
    run, peak = abi.bispec_workspace_bytes(cfg)
    # every grid class keeps the float32 fields of its shell range on its grid;
    # planning holds the float64 unit shells of one class at a time
    grids, lo, hi, _ = abi.bispec_grid_classes(cfg)
    f32 = sum((h - l + 1) * g ** 3 * 4 for g, l, h in zip(grids, lo, hi))
    f64 = max((h - l + 1) * g ** 3 * 8 for g, l, h in zip(grids, lo, hi))
    assert run > f32 and peak > f64
    assert run < 1.2 * f32 + 5e9 and peak < 1.2 * max(f32, f64) + 10e9
    run512, peak512 = abi.bispec_workspace_bytes(abi.make_config(512, 1500.0, 1.0, 100, rsd_beta=0.5, n_est=512)[0])
    assert run512 > 100 * 512 ** 3 * 4 and peak512 > 100 * 512 ** 3 * 8
    assert run512 < 80e9 and peak512 < 150e9


def test_estimator_grid():
    """G is the smallest supported size above 3 max|m_i| (the largest mode
    component is floor(sqrt(hi2 - 1)) of the outermost shell), at most n_g."""
    def grid(*a, **kw):
        return abi.bispec_estimator_grid(abi.make_config(*a, **kw)[0])
    # 100 shells of width 1: max component 100 -> G > 300 -> 320 (5 * 64)
    assert grid(512, 1500.0, 1.0, 100) == 320
    assert grid(1024, 1500.0, 1.0, 100) == 320
    # 10 shells of width 1: max 10 -> G > 30 -> 32
    assert grid(64, 300.0, 1.0, 10) == 32
    assert grid(32, 300.0, 1.0, 10) == 32
    # 40 shells of width 2: top edge 81, max component 80 -> G > 240 -> 256
    assert grid(256, 1000.0, 2.0, 40) == 256
    # 4 shells of width 1 (max 4): G > 12 -> 16; 2 shells (max 2): the smallest grid, 8
    assert grid(96, 100.0, 1.0, 4) == 16
    assert grid(96, 100.0, 1.0, 2) == 8
    assert grid(512, 1500.0, 1.0, 100, n_est=384) == 384
    assert grid(512, 1500.0, 1.0, 100, n_est=512) == 512
    for bad in (256, 300, 640):   # too small, unsupported, above n_g
        with pytest.raises(abi.BispecError) as e:
            grid(512, 1500.0, 1.0, 100, n_est=bad)
        assert e.value.status == abi.BISPEC_EINVAL


def test_no_workspace_flag_on_the_host():
    """BISPEC_FLAG_NO_WORKSPACE plans keep only their tables (run bytes far
    below a plan with a workspace) and exclude GRAD and AUTOTUNE."""
    import paper_2107_14564_amd as P
    c_own, _ = P.make_config(64, 300.0, 1.0, 20)
    c_none, _ = P.make_config(64, 300.0, 1.0, 20, flags=P.FLAG_NO_WORKSPACE)
    own = P.bispec_workspace_bytes(c_own)[0]
    none = P.bispec_workspace_bytes(c_none)[0]
    assert none < own / 100
    for extra in (P.FLAG_GRAD, P.FLAG_AUTOTUNE):
        c_bad, _ = P.make_config(64, 300.0, 1.0, 20, flags=P.FLAG_NO_WORKSPACE | extra)
        with pytest.raises(P.BispecError) as e:
            P.bispec_workspace_bytes(c_bad)
        assert e.value.status == -1


def test_grid_classes_of_the_headline_plan():
    """Every triangle sits in a class whose grid is exact for it
    (G > R_a1 + R_a2 + R_a3 and G > 2 R_a1, R_n = n for shells of width k_f) and
    whose shell range covers its shells; the largest grid is the estimator
    grid; forcing n_est or FLAG_ONE_GRID gives one class on that grid."""
    cfg = abi.make_config(512, 1500.0, 1.0, 100, rsd_beta=0.5)[0]
    tri = np.array(abi.bispec_query_triangles(cfg)[0])
    grids, lo, hi, tc = abi.bispec_grid_classes(cfg)
    tc = np.array(tc)
    assert grids == sorted(grids) and grids[-1] == abi.bispec_estimator_grid(cfg) == 320
    assert len(grids) > 1 and set(tc.tolist()) == set(range(len(grids)))
    g = np.array(grids)[tc]
    assert np.all(g > tri.sum(1)) and np.all(g > 2 * tri[:, 0])
    assert np.all(tri[:, 2] >= np.array(lo)[tc]) and np.all(tri[:, 0] <= np.array(hi)[tc])
    for one in (abi.make_config(512, 1500.0, 1.0, 100, n_est=384)[0],
                abi.make_config(512, 1500.0, 1.0, 100, flags=abi.FLAG_ONE_GRID)[0]):
        grids1, lo1, hi1, tc1 = abi.bispec_grid_classes(one)
        assert len(grids1) == 1 and lo1 == [1] and hi1 == [100] and set(tc1) == {0}
    assert abi.bispec_grid_classes(abi.make_config(512, 1500.0, 1.0, 100, n_est=384)[0])[0] == [384]
