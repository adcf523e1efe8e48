"""Throughput of the FFT bispectrum estimator on one MI355X.

One step = one full pass of the estimator (forward R2C FFT, per-shell inverse
FFTs, triple contraction, float64 normalisation) over the synthetic field of
the workload, with the field already resident in HBM.

Default workload: N_g = 512, L = 1500 Mpc, P(k) = k^-1.5, f_NG = 2, linear RSD
beta = 0.5 along z, 100 shells of width one k_f, all 89 625 closable
triangles, split-bf16 MFMA contraction.

Prints one JSON line (rank 0): metric/value/unit, the per-stage times, the
roofline of the dominant kernel (the contraction) measured with HIP events
recorded by the library on the run stream, the plain-fp32 contraction time of
the same plan, and the float64 CPU oracle timed on a bounded sample.

The roofline's `traffic` (HBM bytes per launch of the contraction) comes from
the rocprofv3 FETCH_SIZE / WRITE_SIZE summary committed under profiles/; it is
reported only while the contraction sources hash to the value recorded there
(else null).  --copy-calibration adds a plain 1 GiB device copy after the timed
region: its counter readings give the bytes-per-count scale of those runs.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (synth workload key, n_g, box_l, dk, n_shells, rsd_beta, selection)
    "ng512_100shells_rsd": dict(field="ng512", n_g=512, box_l=1500.0, dk=1.0, n_shells=100, rsd_beta=0.5, sel={}),
    # the same estimator on a 1024^3 grid (the paper's largest timing point is N_g = 1000)
    "ng1024_100shells_rsd": dict(field="ng1024", n_g=1024, box_l=3000.0, dk=1.0, n_shells=100, rsd_beta=0.5,
                                 sel={}),
    "ng256_40shells_grid": dict(field="ng256", n_g=256, box_l=1000.0, dk=2.0, n_shells=40, rsd_beta=0.0,
                                sel=dict(tri_mode=2, k1_shells=list(range(2, 41, 2)), n_mu=20, n_t=20)),
    "ng32_10shells_grid": dict(field="ng32", n_g=32, box_l=300.0, dk=1.0, n_shells=10, rsd_beta=0.0,
                               sel=dict(tri_mode=2, k1_shells=list(range(5, 11)), n_mu=10, n_t=10)),
    # voxel-slab streaming: 1024^3, shells of 2 k_f, 128 shells, all 185 056 bins (whole fields do not fit)
    "ng1024_w2_128shells_stream": dict(field="ng1024", n_g=1024, box_l=3000.0, dk=2.0, n_shells=128, rsd_beta=0.5,
                                       sel={}),
    # the redshift-space quadrupole (Section 3.1, Legendre weight on the first side): 60 shells at 512^3
    "ng512_60shells_rsd_quadrupole": dict(field="ng512", n_g=512, box_l=1500.0, dk=1.0, n_shells=60, rsd_beta=0.5,
                                          sel=dict(ell=2)),
    # the fourth-order polyspectrum (Section 4): all 35 345 bins of 30 shells on a 128^3 grid
    "ng128_30shells_order4": dict(field="ng128", n_g=128, box_l=600.0, dk=1.0, n_shells=30, rsd_beta=0.5,
                                  sel=dict(order=4)),
    # differentiation workload: 30 shells, a1 in {29, 30} (494 triangles); --grad times bispec_grad too
    "ng256_30shells_grad": dict(field="ng256_grad", n_g=256, box_l=1000.0, dk=1.0, n_shells=30, rsd_beta=0.0,
                                sel=dict(tri_mode=1, k1_shells=[29, 30])),
}

# batched form: 64 heterogeneous realisations (N_g in {96, 128, 160}, 16-48 shells)
BATCH_WORKLOADS = {"batch64_ng96_160": dict(n=64, seed=4999),
                   # the validation ensemble: 32 realisations of one configuration per replay
                   "ensemble32_ng64": dict(n=32, ensemble=dict(n_g=64, box_l=600.0, n_shells=20, k1_shells=[16, 17, 18, 19, 20],
                                                          seed=11000))}

PEAK_BF16_TFLOPS = 2500.0   # MI355X dense bf16 MFMA
PEAK_FP32_VALU_TFLOPS = 78.6   # MI355X fp32 vector FMAs without packed forms (not used in this build)
PEAK_HBM_GBS = 8000.0
TARGET_MFMA_FRAC = 0.5         # contraction target: half of the bf16 MFMA peak
TARGET_SPEEDUP_VS_FP32 = 3.0   # split-bf16 contraction against the plain fp32 one

# sources that determine the contraction kernel and its launch (tiling, ranges)
TRAFFIC_SOURCES = ["paper_2107_14564_amd/csrc/contract_kernels.hip", "paper_2107_14564_amd/csrc/geometry.cpp",
                   "paper_2107_14564_amd/csrc/geometry.h", "paper_2107_14564_amd/csrc/kernels.h",
                   "paper_2107_14564_amd/csrc/api.cpp"]


def contraction_source_hash() -> str:
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload: str):
    """HBM bytes per launch of the split-bf16 contraction from the committed
    counter summary, or None if absent or taken from other sources."""
    path = os.path.join(ROOT, "profiles", "traffic_k_contract_bf16x3_%s.md" % workload)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_sha = re.search(r"^source_sha256:\s*([0-9a-f]{64})\s*$", txt, re.M)
    m_b = re.search(r"^hbm_bytes_per_launch:\s*([0-9.eE+]+)\s*$", txt, re.M)
    if not (m_sha and m_b) or m_sha.group(1) != contraction_source_hash():
        return None
    return float(m_b.group(1))


def copy_calibration(torch, dev, n_bytes: int = 1 << 30, reps: int = 3):
    """A plain streaming copy (read n_bytes, write n_bytes) for counter scaling."""
    src = torch.ones(n_bytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(reps):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    return {"bytes_read": n_bytes, "bytes_written": n_bytes, "launches": reps, "kernel": "torch.neg (elementwise)"}


def class_work(plan, tri):
    """Algorithmic work of a plan's contraction and shell transforms: each
    triangle's triple sum runs over its grid class's G_c^3 points (2 G_c^3 flop,
    plus G_c^3 per distinct (a1, a2) pair product of the class); the shell
    transforms write n_s,c G_c^3 field values per class."""
    import numpy as np
    tc = plan.tri_class.numpy()
    flop, field_vox = 0.0, 0.0
    for k, (g, lo, hi) in enumerate(zip(plan.class_grids, plan.class_shell_lo, plan.class_shell_hi)):
        t = tri[tc == k]
        # order 4: T = sum P_(a1,a2) P_(a3,a4), pairs from both halves of each bin
        pairs = {(int(r[0]), int(r[1])) for r in t} | ({(int(r[2]), int(r[3])) for r in t} if t.shape[1] == 4 else set())
        flop += float(g) ** 3 * (2.0 * len(t) + len(pairs))
        # a multipole plan writes a weighted copy of every class shell as well
        field_vox += float(g) ** 3 * (hi - lo + 1) * (2 if getattr(plan, "ell", 0) else 1)
    return flop, field_vox


def cpu_baseline(delta32, w: dict, plan_tri, plan_ntri, b_gpu, ell: int = 0) -> tuple:
    """The float64 oracle on a bounded sample of the same workload: all closable
    triangles of the first S shells at the full grid (forward FFT, S data and S
    unit shells, the triple sums and their summation scale, N_tri).  Returns the
    baseline record and the timed GPU run's error on those triangles against it
    (e_norm, max e_cond, N_tri equality)."""
    import numpy as np

    from oracle import fbe, geometry, multipoles, polyspectrum
    cores = os.cpu_count() or 1
    d64 = delta32.astype(np.float64)
    t0 = time.perf_counter()
    if plan_tri.shape[1] == 4:
        s_shells = w["n_shells"]   # every quadruple of the workload (30 shells: 60 float64 fields of 128^3, ~12 s)
        tri = polyspectrum.all_quads(s_shells)
        ref = polyspectrum.fft_estimate(d64, w["box_l"], w["dk"], tri, rsd_beta=w["rsd_beta"], with_abs=True)
        ref = {"B": ref["T4"], "S": ref["S"], "ntri": ref["nquad"]}
        what, unit = "quadruples", "quadruples/s"
    else:
        s_shells = 6 if delta32.shape[0] <= 512 else 2   # 12 (4) float64 fields of N^3 on the host, ~10 s
        tri = geometry.all_triangles(s_shells)
        if ell:
            ref = multipoles.estimate(d64, w["box_l"], w["dk"], tri, ell, rsd_beta=w["rsd_beta"], with_abs=True)
        else:
            ref = fbe.estimate(d64, w["box_l"], w["dk"], tri, rsd_beta=w["rsd_beta"], with_abs=True)
        what, unit = "triangles", "triangles/s"
    dt = time.perf_counter() - t0
    base = {"value": len(tri) / dt, "unit": unit, "cores": cores, "kind": "oracle",
            "sample": "all %d closable %s of shells 1-%d at N_g=%d (float64 FFTs, fields, multiple sums "
                      "and their summation scale, bin counts) in %.2f s" % (len(tri), what, s_shells,
                                                                           delta32.shape[0], dt),
            "seconds": dt}
    index = {tuple(int(v) for v in r): t for t, r in enumerate(plan_tri)}
    idx = np.array([index.get(tuple(int(v) for v in r), -1) for r in tri])
    if np.any(idx < 0):
        return base, None
    b = b_gpu[idx]
    err = {"vs": "float64 oracle", "n_checked": int(len(tri)),
           "e_norm": float(np.linalg.norm(b - ref["B"]) / np.linalg.norm(ref["B"])),
           "e_cond": float(np.max(np.abs(b - ref["B"]) / ref["S"])),
           "e_strict_max": float(np.max(np.abs(b - ref["B"]) / np.abs(ref["B"]))),
           "ntri_exact": bool(np.array_equal(plan_ntri[idx], ref["ntri"]))}
    return base, err


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="ng512_100shells_rsd", choices=sorted(WORKLOADS) + sorted(BATCH_WORKLOADS))
    ap.add_argument("--autotune", action="store_true", help="plan with FLAG_AUTOTUNE")
    ap.add_argument("--grad", action="store_true", help="also time the vector-Jacobian product (bispec_grad)")
    ap.add_argument("--precision", default="splitbf16", choices=["splitbf16", "fp32"])
    ap.add_argument("--no-fp32-compare", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (the estimator would shard "
              "voxel slabs across GPUs and add the partial triple sums).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2107_14564_amd as P
    from synth import workload_field

    if args.workload in BATCH_WORKLOADS:
        return bench_batch(args, np, torch, P)
    w = WORKLOADS[args.workload]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    delta32 = np.ascontiguousarray(workload_field(w["field"]), dtype=np.float32)
    gen_s = time.perf_counter() - t0
    print("field ready (%.1f s)" % gen_s, file=sys.stderr, flush=True)
    delta = torch.from_numpy(delta32).to(dev)
    prec = P.PREC_SPLITBF16 if args.precision == "splitbf16" else P.PREC_FP32
    t0 = time.perf_counter()
    plan = P.Plan(w["n_g"], w["box_l"], w["dk"], w["n_shells"], rsd_beta=w["rsd_beta"], precision=prec,
                  flags=P.FLAG_STAGE_TIMING | (P.FLAG_AUTOTUNE if args.autotune else 0) |
                  (P.FLAG_GRAD if args.grad else 0), **w["sel"])
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    print("plan ready (%.1f s), %d triangles" % (plan_s, plan.n_tri), file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        plan.run(delta)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stages = np.zeros(4)
    step_ms = []
    for k in range(args.steps):
        start.record(stream)
        B = plan.run(delta)
        stop.record(stream)
        stop.synchronize()
        step_ms.append(start.elapsed_time(stop))
        stages += np.array(plan.stage_times())
        print("step %d: %.3f ms" % (k, step_ms[-1]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    stages /= args.steps
    ms = float(np.mean(step_ms))
    b_host = B.cpu().numpy()
    assert np.all(np.isfinite(b_host)), "non-finite B"

    n = w["n_g"]
    g = plan.n_est
    tri = plan.triangles.numpy()
    flop, field_vox = class_work(plan, tri)
    # a streamed plan runs the contraction slab by slab between the shell
    # passes: its contraction stage is then folded into the shell stage
    streamed = plan.slabs > 1
    contract_ms = float(stages[1] + stages[2]) if streamed else float(stages[2])
    achieved = flop / (contract_ms * 1e-3) / 1e12
    order4 = plan.order == 4
    unit = "quadruples/s" if order4 else "triangles/s"
    kernel = ("k_contract4<false>" if order4 else "k_contract_bf16x3") if prec == P.PREC_SPLITBF16 \
        else "k_contract_vec<float>"
    result = {
        "metric": unit,
        "value": plan.n_tri / (ms * 1e-3),
        "unit": unit,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3-fp32acc" if prec == P.PREC_SPLITBF16 else "fp32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_g": n, "n_est": g, "box_l": w["box_l"], "n_shells": w["n_shells"],
                   "dk_kf": w["dk"], "rsd_beta": w["rsd_beta"], "n_tri": plan.n_tri, "precision": args.precision,
                   "ell": plan.ell, "order": plan.order},
        "stages_ms": {"forward_fft": stages[0], "shell_ffts": stages[1], "contraction": stages[2],
                      "normalise": stages[3]},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_BF16_TFLOPS,
                     "traffic": measured_traffic(args.workload) if prec == P.PREC_SPLITBF16 and not order4
                     else None,
                     "kernel": kernel + (" (streamed: with the y and z shell passes)" if streamed else ""),
                     "algorithmic_flop": flop},
        "grid_classes": [dict(grid=gc, shells=[lo, hi], n_tri=int((plan.tri_class.numpy() == k).sum()),
                              n_krange=cp["n_krange"], max_cols=cp["max_cols"], n_wg=cp["n_wg"],
                              rep=cp["rep"], tune=cp["tune_source"])
                         for k, (gc, lo, hi, cp) in enumerate(zip(plan.class_grids, plan.class_shell_lo,
                                                                  plan.class_shell_hi, plan.classes()))],
        "fft_hbm": {"algorithmic_bytes": (8.0 * n ** 3 + 4.0 * field_vox),
                    "achieved_GBs": (8.0 * n ** 3 + 4.0 * field_vox) / ((stages[0] + stages[1]) * 1e-3) / 1e9,
                    "peak_GBs": PEAK_HBM_GBS},
        "plan_s": plan_s,
        "x_slabs_per_class": plan.slabs,
    }
    # the paper's cost unit: mode triangles (sum of N_tri over the bins) per second; mode
    # quadruples (sum of N_quad) for the fourth order
    result["mode_quadruples_per_s" if order4 else "mode_triangles_per_s"] = (
        float(plan.ntri.numpy().astype(np.float64).sum()) / (ms * 1e-3))
    result["fft_hbm"]["frac"] = result["fft_hbm"]["achieved_GBs"] / PEAK_HBM_GBS
    if streamed:  # the shell stage holds the contraction too: no FFT-only rate
        result["fft_hbm"] = None
    if not args.no_fp32_compare and prec == P.PREC_SPLITBF16 and not order4 and not streamed:
        plan.set_precision(P.PREC_FP32)
        plan.run(delta)
        torch.cuda.synchronize()
        f32 = []
        for _ in range(max(2, min(3, args.steps))):
            plan.run(delta)
            torch.cuda.synchronize()
            f32.append(plan.stage_times()[2])
        b32 = plan.run(delta).cpu().numpy()
        plan.set_precision(prec)
        result["fp32_contraction_ms"] = float(np.mean(f32))
        result["speedup_vs_fp32_contraction"] = float(np.mean(f32)) / contract_ms
        # the fp32 form at the fp32 vector peak would take flop / 78.6 TFLOP/s
        result["fp32_floor_ms"] = flop / (PEAK_FP32_VALU_TFLOPS * 1e12) * 1e3
        result["speedup_vs_fp32_floor"] = result["fp32_floor_ms"] / contract_ms
        result["splitbf16_vs_fp32_norm_diff"] = float(np.linalg.norm(b_host - b32) / np.linalg.norm(b32))
        result["targets"] = {
            "contraction_mfma_frac": {"target": TARGET_MFMA_FRAC, "achieved": achieved / PEAK_BF16_TFLOPS,
                                      "met": achieved / PEAK_BF16_TFLOPS >= TARGET_MFMA_FRAC},
            "speedup_vs_fp32": {"target": TARGET_SPEEDUP_VS_FP32, "measured": result["speedup_vs_fp32_contraction"],
                                "vs_fp32_floor": result["speedup_vs_fp32_floor"],
                                "met": result["speedup_vs_fp32_floor"] >= TARGET_SPEEDUP_VS_FP32}}
    if args.grad:
        # vector-Jacobian product of the last run: adjoint field build, pruned
        # forward transforms of every adjoint shell, one inverse at n_g
        g_b = torch.ones(plan.n_tri, dtype=torch.float64, device=dev)
        plan.grad(g_b)
        torch.cuda.synchronize()
        gms = []
        for _ in range(max(2, min(5, args.steps))):
            start.record(stream)
            plan.grad(g_b)
            stop.record(stream)
            stop.synchronize()
            gms.append(start.elapsed_time(stop))
        result["grad_ms"] = float(np.mean(gms))
        # algorithmic bytes of the adjoint: read every class field once (G build,
        # 4 B per field value), write G (4 B), the forward transforms read G
        # (4 B), the last inverse writes gdelta (4 N^3)
        gbytes = 12.0 * field_vox + 4.0 * float(n) ** 3
        result["grad_hbm"] = {"algorithmic_bytes": gbytes, "achieved_GBs": gbytes / (result["grad_ms"] * 1e-3) / 1e9,
                              "peak_GBs": PEAK_HBM_GBS}
    if args.copy_calibration:
        result["copy_calibration"] = copy_calibration(torch, dev)
    if not args.no_cpu_baseline:
        print("cpu baseline ...", file=sys.stderr, flush=True)
        result["cpu_baseline"], result["error_vs_oracle"] = cpu_baseline(delta32, w, tri, plan.ntri.numpy(), b_host,
                                                                          plan.ell)
    plan.close()
    print(json.dumps(result), flush=True)


def bench_batch(args, np, torch, P):
    """The batched form: every member of the ensemble in one replay of a captured
    HIP graph; one step = one pass over all members."""
    from synth import batch_field, batch_members
    bw = BATCH_WORKLOADS[args.workload]
    ens = bw.get("ensemble")
    if ens:  # identical configurations, seeded realisations of the quadratic field (f_NG = 1)
        members = [dict(n_g=ens["n_g"], box_l=ens["box_l"], n_shells=ens["n_shells"], f_ng=1.0,
                        seed=ens["seed"] + i) for i in range(bw["n"])]
    else:
        members = batch_members(bw["n"], bw["seed"])
    prec = P.PREC_SPLITBF16 if args.precision == "splitbf16" else P.PREC_FP32
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    fields = [torch.from_numpy(np.ascontiguousarray(batch_field(m), dtype=np.float32)) for m in members]
    print("fields ready (%.1f s)" % (time.perf_counter() - t0), file=sys.stderr, flush=True)
    sel = dict(tri_mode=P.TRI_K1SET, k1_shells=ens["k1_shells"]) if ens else {}
    configs = [dict(n_g=m["n_g"], box_l=m["box_l"], dk=1.0, n_shells=m["n_shells"], precision=prec,
                    flags=P.FLAG_AUTOTUNE if args.autotune else 0, **sel) for m in members]
    t0 = time.perf_counter()
    bp = P.BatchPlan(configs)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    print("batch plan ready (%.1f s), %d triangles" % (plan_s, bp.n_tri), file=sys.stderr, flush=True)
    packed = bp.pack(fields)
    out = torch.empty(bp.n_tri, dtype=torch.float64, device=dev)
    for _ in range(max(1, args.warmup)):
        bp.run_into(packed, out, use_graph=True)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    step_ms = []
    for k in range(args.steps):
        start.record(stream)
        bp.run_into(packed, out, use_graph=True)
        stop.record(stream)
        stop.synchronize()
        step_ms.append(start.elapsed_time(stop))
        print("step %d: %.3f ms" % (k, step_ms[-1]), file=sys.stderr, flush=True)
    ms = float(np.mean(step_ms))
    assert np.all(np.isfinite(out.cpu().numpy())), "non-finite B"
    # direct launches of the same batch, for the graph's gain
    bp.run(packed, use_graph=False)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(max(1, min(3, args.steps))):
        bp.run(packed, use_graph=False)
    stop.record(stream)
    stop.synchronize()
    eager_ms = start.elapsed_time(stop) / max(1, min(3, args.steps))
    # the grid classes and the autotuner's choices, over all members
    tuning = {}
    for i in range(bp.n):
        for c in bp.classes(i):
            key = "G%d_cols%d_ranges%d_%s" % (c["grid"], c["max_cols"], c["n_krange"], c["tune_source"])
            tuning[key] = tuning.get(key, 0) + 1
    flop = 0.0
    for i in range(bp.n):
        tri = bp.triangles[i].numpy()
        grids, _, _, tc = P.bispec_grid_classes(bp_cfg(P, configs[i]))
        tc = np.array(tc)
        for k, g in enumerate(grids):
            t = tri[tc == k]
            n_pairs = len({(int(a), int(b)) for a, b, _ in t})
            flop += float(g) ** 3 * (2.0 * len(t) + n_pairs)
    achieved = flop / (ms * 1e-3) / 1e12
    result = {
        "metric": "triangles/s", "value": bp.n_tri / (ms * 1e-3), "unit": "triangles/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16x3-fp32acc" if prec == P.PREC_SPLITBF16 else "fp32", "data": "synthetic",
        "config": {"workload": args.workload, "members": bp.n, "grids": sorted({m["n_g"] for m in members}),
                   "n_shells_range": [min(m["n_shells"] for m in members), max(m["n_shells"] for m in members)],
                   "n_tri": bp.n_tri, "precision": args.precision, "autotune": bool(args.autotune)},
        "eager_ms_per_step": eager_ms,
        "contraction_launches_per_step": 1,
        "class_tuning": tuning,
        "realisations_per_s": bp.n / (ms * 1e-3),
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_BF16_TFLOPS, "traffic": None, "kernel": "whole step (all kernels)",
                     "algorithmic_flop": flop},
        "plan_s": plan_s,
    }
    if not args.no_cpu_baseline:
        result["error_vs_oracle"] = batch_error(bp, fields, configs, out.cpu().numpy(), np)
    bp.close()
    print(json.dumps(result), flush=True)


def batch_error(bp, fields, configs, b_all, np) -> dict:
    """The timed batch's error against the float64 oracle on a bounded sample:
    for the first and the last member, its bins of the six smallest first sides
    (at most 200), on the member's full grid."""
    from oracle import fbe
    members = sorted({0, bp.n - 1})
    d2 = r2 = 0.0
    e_cond = 0.0
    n_checked = 0
    ntri_ok = True
    for i in members:
        c = configs[i]
        tri = bp.triangles[i].numpy()
        pick = np.where(tri[:, 0] <= tri[:, 0].min() + 5)[0][:200]
        ref = fbe.estimate(fields[i].numpy().astype(np.float64), c["box_l"], c["dk"], tri[pick], rsd_beta=0.0,
                           with_abs=True)
        got = b_all[bp.b_off[i]:bp.b_off[i + 1]][pick]
        d2 += float(np.sum((got - ref["B"]) ** 2))
        r2 += float(np.sum(ref["B"] ** 2))
        e_cond = max(e_cond, float(np.max(np.abs(got - ref["B"]) / ref["S"])))
        ntri_ok = ntri_ok and bool(np.array_equal(bp.ntri[i].numpy()[pick], ref["ntri"]))
        n_checked += len(pick)
    return {"vs": "float64 oracle", "members": members, "n_checked": n_checked,
            "sample": "the bins of the six smallest first sides of each sampled member (at most 200), full grid",
            "e_norm": (d2 / r2) ** 0.5 if r2 > 0 else None, "e_cond": e_cond, "ntri_exact": ntri_ok}


def bp_cfg(P, c):
    c = dict(c)
    return P.make_config(c.pop("n_g"), c.pop("box_l"), c.pop("dk"), c.pop("n_shells"), **c)[0]


if __name__ == "__main__":
    main()
