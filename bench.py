#!/usr/bin/env python3
"""Benchmark of the surrogate-matrix assembly path on one MI355X.

Step: one surrogate assembly (FP64, M = 8, q = 3) of the 3D p = 3 Poisson
stiffness on the sine-mapped unit cube with 128^3 elements (131^3 dofs,
343-slot stencils): quadrature of the boundary and sample rows, spline fit,
fill of every other row, padding.  The step executes a kept assembly plan
(igs_plan_*: host-side tables and the geometry check made once), so each step
is the assembly's GPU work; the one-shot call (plan built and freed per call,
synchronising) is timed separately.  value = band slots assembled per second
(N * S / step time).  The same run also measures, each with its own timing,
full quadrature assembly of the same matrix, the banded SpMV, CG in FP64 and
FP32-inside-FP64-refinement to 1e-10, the batched 2D compliance solve +
adjoint, and the 2D p = 2, q = 5 timing study with mesh-dependent sampling
lengths; those figures go into the same JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extra] [--copy-probe]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6

# HBM bytes per launch of this workload's kernels from rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE runs (KiB per dispatch), scaled by what the same
# counters give for a plain 2^30-byte elementwise copy (FETCH 2.00, WRITE 1.00);
# profiles/*_hbm_counters.md hold the runs (keys: phase names of the domain
# surrogate step, fe_* of the face/edge step, mf_* of the matrix-free apply,
# pd_fill of the per-delta step).
# A figure is only reported while the kernel sources still hash to the ones
# measured.
PMC_FETCH_SCALE, PMC_WRITE_SCALE = 2.00, 1.00
PMC_TRAFFIC = {
    "quad_boundary_rows": {"sources": ["quad.hip", "plan.cpp"], "sha256": "a5c4085700c26a0f", "fetch_kib": 14977.6, "write_kib": 2429550.5},
    "fill": {"sources": ["fill.hip"], "sha256": "a839a6953e4cbe7c", "fetch_kib": 152703.5, "write_kib": 4971999.7},
    "diag_fixup": {"sources": ["fill.hip"], "sha256": "a839a6953e4cbe7c", "fetch_kib": 361340.0, "write_kib": 2612.8},
    "fe_fill": {"sources": ["fill.hip", "plan.cpp"], "sha256": "6407a3d7e3a2617e", "fetch_kib": 946652.3, "write_kib": 6024184.5},
    "fe_quad_rows": {"sources": ["quad.hip", "plan.cpp"], "sha256": "a5c4085700c26a0f", "fetch_kib": 2133.6, "write_kib": 128203.9},
    "fe_quad_tiles": {"sources": ["quad.hip", "plan.cpp"], "sha256": "a5c4085700c26a0f", "fetch_kib": 682.5, "write_kib": 39873.8},
    "mf_domain_rows": {"sources": ["fill.hip"], "sha256": "a839a6953e4cbe7c", "fetch_kib": 117030.8, "write_kib": 13497.2},
    "mf_copied_entries": {"sources": ["fill.hip"], "sha256": "a839a6953e4cbe7c", "fetch_kib": 396878.9, "write_kib": 2612.8},
    "mf_stored_rows": {"sources": ["fill.hip"], "sha256": "a839a6953e4cbe7c", "fetch_kib": 1018429.4, "write_kib": 4820.7},
    "pd_fill": {"sources": ["fillpd.hip", "plan.cpp"], "sha256": "2eb2fe809d26d3e7", "fetch_kib": 98490.9, "write_kib": 5143617.4},
}


def source_hash(sources):
    import hashlib

    h = hashlib.sha256()
    for src in sources:
        h.update(open(os.path.join(ROOT, "paper_1904_06971_amd", "csrc", src), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(phase):
    """Scaled HBM bytes per launch for a phase, or None when not measured for
    the kernel sources (and tile planner) as they are now."""
    rec = PMC_TRAFFIC.get(phase)
    if rec is None or source_hash(rec["sources"]) != rec["sha256"]:
        return None
    return (rec["fetch_kib"] * PMC_FETCH_SCALE + rec["write_kib"] * PMC_WRITE_SCALE) * 1024.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def quad_flops_per_row(n, p):
    """Algorithmic flops of sum-factorised row quadrature (stiffness): per
    (a, b) component (p+1)^5 + (2p+1)(p+1)^4 + (2p+1)^2(p+1)^3 FMA in 3D,
    (p+1)^4 + (2p+1)(p+1)^3 in 2D; n^2 components; 2 flops per FMA."""
    if n == 3:
        fma = (p + 1) ** 5 + (2 * p + 1) * (p + 1) ** 4 + (2 * p + 1) ** 2 * (p + 1) ** 3
    else:
        fma = (p + 1) ** 4 + (2 * p + 1) * (p + 1) ** 3
    return 2 * n * n * fma


def fill_bytes(prob, lay, esize):
    """Algorithmic HBM bytes of the fill and copy kernels.  The fill writes
    every slot of every analysis-domain row once (it reads nothing of the
    band); the copy kernel reads and writes each copied exact entry (partner
    outside the analysis domain) once and updates the diagonal of each row
    that has one."""
    n, p = prob["n"], prob["p"]
    L = [lay.m[d] - 4 * p for d in range(n)]
    rows = math.prod(L)
    both = math.prod(sum(L[d] - abs(dl) for dl in range(-p, p + 1)) for d in range(n))
    copies = rows * lay.slots - both
    shell = rows - math.prod(max(0, L[d] - 2 * p) for d in range(n))
    return rows * lay.slots * esize, rows, copies, (2 * copies + 2 * shell) * esize, shell


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="only the timed step (for profiling runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (reference kernel for HBM byte counters)")
    ap.add_argument("--leg", choices=["face_edge", "per_delta", "matrix_free"], default=None,
                    help="only run one other leg's timed steps on the same workload (for profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the path runs on a single GPU (sharding is described in the "
              "design notes, not implemented); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1904_06971_amd import igs
    from paper_1904_06971_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe:
        # a plain elementwise kernel that reads and writes 2^30 bytes once each:
        # the reference for scaling the profiler's FETCH_SIZE / WRITE_SIZE counts
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 1 << 30, "kernel": "neg (elementwise)", "launches": 3}), flush=True)
        return
    if args.leg:
        profile_leg(args)
        return
    prob = W.c4_precision3d()
    M, q = 8, 3
    lay = igs.layout(prob)
    info, _ = igs.surrogate_layout(prob, M, q)
    slots = lay.N * lay.slots
    true_nnz = math.prod(lay.m[d] * (2 * prob["p"] + 1) - prob["p"] * (prob["p"] + 1) for d in range(3))
    band = igs.empty_band(prob, torch.float64)
    stream = torch.cuda.current_stream()

    # ------------------------------------------------------------ timed step
    # a kept plan (host tables, tile lists and the geometry check made once);
    # every step runs all of the assembly's kernels
    plan = igs.Plan(prob, igs.STIFFNESS, M=M, q=q)
    for _ in range(max(1, args.warmup)):
        plan.execute(out=band)
    torch.cuda.synchronize()
    igs.profile_enable(True)
    igs.profile_read()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        plan.execute(out=band)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = igs.profile_read()
    igs.profile_enable(False)
    ms_step = ev0.elapsed_time(ev1) / args.steps
    value = slots / (ms_step * 1e-3)
    phases = {k: {"launches": v[0], "avg_ms": v[1] / v[0]} for k, v in prof.items()}
    log(f"surrogate: {ms_step:.3f} ms/step (wall {wall / args.steps * 1e3:.3f}), {value:.3e} slots/s, phases {phases}")
    # the same number of steps again, each between its own events: median and spread
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    evs[0].record(stream)
    for k in range(args.steps):
        plan.execute(out=band)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    per_step = sorted(evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps))
    step_stats = {"median_ms": per_step[len(per_step) // 2] if len(per_step) % 2 else
                  0.5 * (per_step[len(per_step) // 2 - 1] + per_step[len(per_step) // 2]),
                  "min_ms": per_step[0], "max_ms": per_step[-1], "steps": args.steps}
    log(f"per-step: {step_stats}")

    # rooflines of the step's kernels
    fpr = quad_flops_per_row(3, prob["p"])
    fb, frows, fcopies, cb, cshell = fill_bytes(prob, lay, 8)
    roofs = {}
    for name, rows in (("quad_boundary_rows", info.boundary_rows), ("quad_sample_rows", info.sample_rows)):
        if name in phases:
            t = phases[name]["avg_ms"] * 1e-3
            tf = fpr * rows / t / 1e12
            roofs[name] = {"bound": "alu", "achieved": tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": tf / FP64_PEAK_TFLOPS, "traffic": measured_traffic(name),
                           "units": f"{rows} quadrature rows", "ms": t * 1e3}
    if "fill" in phases:
        t = phases["fill"]["avg_ms"] * 1e-3
        roofs["fill"] = {"bound": "hbm", "achieved": fb / t / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": fb / t / 1e9 / HBM_PEAK_GBS, "traffic": measured_traffic("fill"), "ms": t * 1e3,
                         "units": f"{frows} analysis-domain rows x {lay.slots} slots"}
    if "copy" in phases:
        t = phases["copy"]["avg_ms"] * 1e-3
        roofs["copy"] = {"bound": "hbm", "achieved": cb / t / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": cb / t / 1e9 / HBM_PEAK_GBS, "traffic": measured_traffic("copy"), "ms": t * 1e3,
                         "units": f"{fcopies} copied entries read and written, {cshell} diagonals updated"}
    if "diag_fixup" in phases:
        # the boundary rows have stored the copied entries (transposed stores);
        # the fix-up reads them from the row's own slots and updates its diagonal
        t = phases["diag_fixup"]["avg_ms"] * 1e-3
        db = (fcopies + 2 * cshell) * 8
        roofs["diag_fixup"] = {"bound": "hbm", "achieved": db / t / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": db / t / 1e9 / HBM_PEAK_GBS, "traffic": measured_traffic("diag_fixup"),
                               "ms": t * 1e3, "units": f"{fcopies} copied entries read, {cshell} diagonals updated"}
    dominant = max(roofs, key=lambda k: roofs[k].get("ms", phases.get(k, {}).get("avg_ms", 0.0)))
    roofline = dict(roofs[dominant])
    roofline["kernel"] = dominant
    # the whole step against the HBM roofline: the band it must write, over the
    # step time (the target reading of ">= 60% of HBM peak" for the assembly)
    band_bytes = slots * 8
    step_hbm = {"bound": "hbm", "achieved": band_bytes / (ms_step * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": band_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "units": f"{slots} band slots x 8 bytes written once", "target_frac": 0.60}
    log(f"whole step: {step_hbm['achieved']:.0f} GB/s algorithmic, {100 * step_hbm['frac']:.1f}% of HBM peak")

    extra = {}
    if not args.no_extra:
        # ------------------------------------- one-shot call (plan built per call)
        igs.assemble_surrogate(prob, igs.STIFFNESS, M, q, out=band)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            igs.assemble_surrogate(prob, igs.STIFFNESS, M, q, out=band)
        torch.cuda.synchronize()
        extra["one_shot_ms"] = (time.perf_counter() - t0) / 5 * 1e3
        log(f"one-shot surrogate call: {extra['one_shot_ms']:.3f} ms")
        # ------------------------------------------- full quadrature assembly
        xplan = igs.Plan(prob, igs.STIFFNESS, M=0, q=0)
        xplan.execute(out=band)
        igs.profile_enable(True)
        igs.profile_read()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(3):
            xplan.execute(out=band)
        e1.record(stream)
        torch.cuda.synchronize()
        pe = igs.profile_read()
        igs.profile_enable(False)
        ms_ex = e0.elapsed_time(e1) / 3
        tq = pe["quad_exact"][1] / pe["quad_exact"][0] * 1e-3
        fl = quad_flops_per_row(3, prob["p"]) * lay.N
        extra["exact_assembly"] = {"ms": ms_ex, "slots_per_s": slots / (ms_ex * 1e-3),
                                   "quad_kernel_tflops": fl / tq / 1e12, "quad_kernel_frac": fl / tq / 1e12 / FP64_PEAK_TFLOPS}
        extra["speedup_surrogate_vs_exact"] = ms_ex / ms_step
        log(f"exact: {ms_ex:.3f} ms; surrogate speed-up {ms_ex / ms_step:.2f}x")
        xplan.close()

        # ------------------------ face/edge stencil functions (Sec. 3.6), same workload
        info_fe = igs.surrogate_fe_layout(prob, M, q)
        fe = {"quadrature_rows": info_fe.quadrature_rows, "domain_surrogate_quadrature_rows": info.quadrature_rows,
              "classes": info_fe.classes}
        for name, tdt, esize in (("f64", torch.float64, 8), ("f32", torch.float32, 4)):
            bfe = band if tdt == torch.float64 else igs.empty_band(prob, tdt)
            pfe = igs.Plan(prob, igs.STIFFNESS, M=M, q=q, dtype=tdt, face_edge=True)
            ms_fe, ph_fe = timed_plan(pfe, bfe, stream, args.steps)
            pfe.close()
            leg = {"ms": ms_fe, "slots_per_s": slots / (ms_fe * 1e-3), "phases_ms": ph_fe,
                   "step_hbm_frac": slots * esize / (ms_fe * 1e-3) / 1e9 / HBM_PEAK_GBS,
                   "fill_hbm_frac": slots * esize / (ph_fe["fill"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
            if name == "f64":
                # the fill writes every slot of every row once (the whole band)
                tf = ph_fe["fill"] * 1e-3
                leg["roofline_fill"] = {"bound": "hbm", "achieved": slots * 8 / tf / 1e9, "peak": HBM_PEAK_GBS,
                                        "unit": "GB/s", "frac": slots * 8 / tf / 1e9 / HBM_PEAK_GBS,
                                        "traffic": measured_traffic("fe_fill"), "ms": ph_fe["fill"],
                                        "units": f"{lay.N} rows x {lay.slots} slots x 8 bytes"}
            if name == "f64":
                leg["speedup_vs_domain_surrogate"] = ms_step / ms_fe
                leg["speedup_vs_exact"] = ms_ex / ms_fe
            fe[name] = leg
            del bfe
        extra["face_edge"] = fe
        log(f"face/edge: {fe}")

        # --------------- per-delta domains (Sec. 4 remark), same workload
        info_pd = igs.surrogate_pd_layout(prob, M, q)
        pdl = {"quadrature_rows": info_pd.quadrature_rows, "noncardinal_rows": info_pd.noncardinal_rows,
               "domain_surrogate_quadrature_rows": info.quadrature_rows,
               "samples_per_direction": list(info_pd.samples)[:3]}
        for name, tdt, esize in (("f64", torch.float64, 8), ("f32", torch.float32, 4)):
            bpd = band if tdt == torch.float64 else igs.empty_band(prob, tdt)
            ppd = igs.Plan(prob, igs.STIFFNESS, M=M, q=q, dtype=tdt, per_delta=True)
            ms_pd, ph_pd = timed_plan(ppd, bpd, stream, args.steps)
            ppd.close()
            leg = {"ms": ms_pd, "slots_per_s": slots / (ms_pd * 1e-3), "phases_ms": ph_pd,
                   "step_hbm_frac": slots * esize / (ms_pd * 1e-3) / 1e9 / HBM_PEAK_GBS}
            if name == "f64":
                # the fill writes the cardinal rows' interpolated slots once
                tf = ph_pd["fill"] * 1e-3
                cb = pd_fill_bytes(prob, lay, esize)
                leg["roofline_fill"] = {"bound": "hbm", "achieved": cb / tf / 1e9, "peak": HBM_PEAK_GBS,
                                        "unit": "GB/s", "frac": cb / tf / 1e9 / HBM_PEAK_GBS,
                                        "traffic": measured_traffic("pd_fill"), "ms": ph_pd["fill"],
                                        "units": "interpolated entries of the cardinal rows plus their diagonals, "
                                                 "8 bytes each"}
                tq = ph_pd["quad_boundary_rows"] * 1e-3
                fl = quad_flops_per_row(3, prob["p"]) * info_pd.noncardinal_rows
                leg["roofline_boundary_rows"] = {"bound": "alu", "achieved": fl / tq / 1e12,
                                                 "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                                                 "frac": fl / tq / 1e12 / FP64_PEAK_TFLOPS, "ms": tq * 1e3,
                                                 "units": f"{info_pd.noncardinal_rows} quadrature rows"}
                leg["speedup_vs_domain_surrogate"] = ms_step / ms_pd
                leg["speedup_vs_exact"] = ms_ex / ms_pd
            pdl[name] = leg
            del bpd
        extra["per_delta"] = pdl
        log(f"per-delta: {pdl}")

        # ------------- 3D p=3 64^3 stiffness and mass, exact vs surrogate M in {4, 8, 16}
        extra["poisson3d_p3_64"] = c2_study(stream, args.steps)
        log(f"3D p=3 64^3: {extra['poisson3d_p3_64']}")

        # -------------------------------------------------------- SpMV / CG
        plan.execute(out=band)
        b32 = igs.assemble_surrogate(prob, igs.STIFFNESS, M, q, dtype=torch.float32)
        # precision form: the same surrogate assembly into FP32 storage (fill and
        # interpolation in FP32), kept plan, timed like the FP64 step
        plan32 = igs.Plan(prob, igs.STIFFNESS, M=M, q=q, dtype=torch.float32)
        plan32.execute(out=b32)
        igs.profile_enable(True)
        igs.profile_read()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(5):
            plan32.execute(out=b32)
        e1.record(stream)
        torch.cuda.synchronize()
        p32 = igs.profile_read()
        igs.profile_enable(False)
        ms32 = e0.elapsed_time(e1) / 5
        extra["fp32_assembly"] = {"ms": ms32, "slots_per_s": slots / (ms32 * 1e-3),
                                  "phases_ms": {k: v[1] / v[0] for k, v in p32.items()},
                                  "fill_GBps": fb / 2 / (p32["fill"][1] / p32["fill"][0] * 1e-3) / 1e9}
        plan32.close()
        log(f"fp32 assembly: {extra['fp32_assembly']}")
        x = torch.randn(1, lay.N, dtype=torch.float64, device=dev)
        x32 = x.float()
        y64, y32 = torch.empty_like(x), torch.empty_like(x32)

        def apply_s(bd, xv, yv, reps=10):
            # back-to-back applications on torch's current stream (the one the
            # library launches on), events around the whole run
            igs.apply(prob, bd, xv, out=yv)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                igs.apply(prob, bd, xv, out=yv)
            e1.record()
            e1.synchronize()
            return e0.elapsed_time(e1) / reps * 1e-3

        t64, t32 = apply_s(band, x, y64), apply_s(b32, x32, y32)
        extra["spmv"] = {"f64_ms": t64 * 1e3, "f64_GBps": lay.slots * lay.N * 8 / t64 / 1e9,
                         "f32_ms": t32 * 1e3, "f32_GBps": lay.slots * lay.N * 4 / t32 / 1e9}
        f = igs.assemble_rhs(prob, igs.SRC_SINE, 3 * math.pi ** 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u64, i64 = igs.solve_cg(prob, band, f, rtol=1e-10, maxit=20000)
        torch.cuda.synchronize()
        tc64 = time.perf_counter() - t0
        t0 = time.perf_counter()
        umx, imx = igs.solve_cg(prob, band, f, band32=b32, rtol=1e-10, maxit=20000)
        torch.cuda.synchronize()
        tcmx = time.perf_counter() - t0
        du = float((umx - u64).abs().max() / u64.abs().max())
        extra["cg"] = {"rtol": 1e-10, "f64_ms": tc64 * 1e3, "f64_iterations": i64["iterations"],
                       "f64_relres": i64["relres"], "mixed_ms": tcmx * 1e3, "mixed_iterations": imx["iterations"],
                       "mixed_outer": imx["outer_iterations"], "mixed_relres": imx["relres"],
                       "mixed_vs_f64_max_rel_diff": du, "speedup_mixed": tc64 / tcmx}
        b32_err = float((b32.double() - band).abs().max() / band.abs().max())
        extra["fp32_band_max_rel_err"] = b32_err
        log(f"cg: {extra['cg']}")
        # matrix-free operator (analysis-domain rows evaluated from the spline
        # coefficients in every product; the band holds only the quadrature rows)
        pmf = igs.Plan(prob, igs.STIFFNESS, M=M, q=q, matrix_free=True)
        ms_mfa, ph_mfa = timed_plan(pmf, band, stream, args.steps)
        ymf = torch.empty_like(x)
        pmf.apply(band, x, dirichlet=True, out=ymf)
        torch.cuda.synchronize()
        igs.profile_enable(True)
        igs.profile_read()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(10):
            pmf.apply(band, x, dirichlet=True, out=ymf)
        e1.record(stream)
        torch.cuda.synchronize()
        pr_mf = igs.profile_read()
        igs.profile_enable(False)
        ms_mf = e0.elapsed_time(e1) / 10
        t0 = time.perf_counter()
        umf, imf = pmf.solve_cg(band, f, rtol=1e-10, maxit=20000)
        torch.cuda.synchronize()
        tcmf = time.perf_counter() - t0
        dmf = float((umf - u64).abs().max() / u64.abs().max())
        pmf.close()
        stored = info.boundary_rows * lay.slots * 8
        dom_rows = lay.N - info.boundary_rows
        flops_mf = dom_rows * lay.slots * (2 * 3 * (q + 1) + 2)
        t_dom = pr_mf["mf_domain_rows"][1] / pr_mf["mf_domain_rows"][0] * 1e-3
        extra["matrix_free"] = {
            "assembly_ms": ms_mfa, "assembly_phases_ms": ph_mfa, "apply_ms": ms_mf,
            "apply_phases_ms": {k: v[1] / v[0] for k, v in pr_mf.items()},
            "banded_apply_ms": t64 * 1e3, "band_bytes_read_per_apply": stored,
            "banded_bytes_read_per_apply": lay.slots * lay.N * 8,
            "domain_rows_roofline": {"bound": "alu", "achieved": flops_mf / t_dom / 1e12, "peak": FP64_PEAK_TFLOPS,
                                     "unit": "TFLOP/s", "frac": flops_mf / t_dom / 1e12 / FP64_PEAK_TFLOPS,
                                     "units": f"{dom_rows} rows x {lay.slots} entries x (2 n (q+1) + 2) flop"},
            "traffic_per_apply": {k: measured_traffic(k) for k in ("mf_domain_rows", "mf_copied_entries",
                                                                   "mf_stored_rows")},
            "cg_ms": tcmf * 1e3, "cg_iterations": imf["iterations"], "cg_relres": imf["relres"],
            "cg_vs_banded_f64_max_rel_diff": dmf, "banded_cg_ms": tc64 * 1e3}
        log(f"matrix-free: {extra['matrix_free']}")
        del ymf, umf
        del b32, x, x32, y64, y32

        # ---------------------------------------- batched 2D compliance + adjoint
        try:
            p5 = W.c5_adjoint2d()
            b5 = igs.assemble_surrogate(p5, igs.STIFFNESS, 8, 3)
            f5 = igs.assemble_rhs(p5, igs.SRC_CONST, 1.0)
            igs.compliance_grad(p5, 8, 3, f5)  # warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b5 = igs.assemble_surrogate(p5, igs.STIFFNESS, 8, 3, out=b5)
            u5, i5 = igs.solve_cg(p5, b5, f5, rtol=1e-10)
            tsolve = time.perf_counter() - t0
            t1 = time.perf_counter()
            g5 = igs.compliance_grad(p5, 8, 3, u5)
            torch.cuda.synchronize()
            tadj = time.perf_counter() - t1
            # the same with the FP32 band inside FP64 residual replacement (both
            # bands assembled inside the timed region; same FP64 stopping test)
            b5f = igs.assemble_surrogate(p5, igs.STIFFNESS, 8, 3, dtype=torch.float32)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            b5 = igs.assemble_surrogate(p5, igs.STIFFNESS, 8, 3, out=b5)
            b5f = igs.assemble_surrogate(p5, igs.STIFFNESS, 8, 3, dtype=torch.float32, out=b5f)
            u5m, i5m = igs.solve_cg(p5, b5, f5, band32=b5f, rtol=1e-10)
            tsolve_m = time.perf_counter() - t2
            t3 = time.perf_counter()
            g5m = igs.compliance_grad(p5, 8, 3, u5m)
            torch.cuda.synchronize()
            tadj_m = time.perf_counter() - t3
            gdiff = float(((g5m - g5).abs().amax(dim=1) / g5.abs().amax(dim=1)).max())
            extra["compliance_2d_batch8"] = {"assembly_cg_ms": tsolve * 1e3, "adjoint_ms": tadj * 1e3,
                                             "cg_plus_adjoint_ms": (tsolve + tadj) * 1e3,
                                             "cg_iterations": i5["iterations"], "relres": i5["relres"],
                                             "mixed": {"assembly_cg_ms": tsolve_m * 1e3, "adjoint_ms": tadj_m * 1e3,
                                                       "cg_plus_adjoint_ms": (tsolve_m + tadj_m) * 1e3,
                                                       "cg_iterations": i5m["iterations"],
                                                       "outer_iterations": i5m["outer_iterations"],
                                                       "relres": i5m["relres"],
                                                       "grad_max_rel_diff_vs_f64": gdiff}}
            del b5, b5f
        except igs.IGSError as e:
            extra["compliance_2d_batch8"] = {"error": str(e)}
        log(f"c5: {extra['compliance_2d_batch8']}")

        # ---------------- 3D p=4 128^3, variable coefficient (kept plans, 2 executions each)
        try:
            p3 = W.c3_varcoef3d()
            lay3 = igs.layout(p3)
            b3 = igs.empty_band(p3, torch.float64)
            c3 = {}
            for name, M3, q3 in (("surrogate", M, q), ("exact", 0, 0)):
                pl3 = igs.Plan(p3, igs.STIFFNESS, M=M3, q=q3)
                pl3.execute(out=b3)
                igs.profile_enable(True)
                igs.profile_read()
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(2):
                    pl3.execute(out=b3)
                e1.record(stream)
                torch.cuda.synchronize()
                pr3 = igs.profile_read()
                igs.profile_enable(False)
                pl3.close()
                ms3 = e0.elapsed_time(e1) / 2
                c3[name] = {"ms": ms3, "slots_per_s": lay3.N * lay3.slots / (ms3 * 1e-3),
                            "phases_ms": {k: v[1] / v[0] for k, v in pr3.items()}}
            fl3 = quad_flops_per_row(3, 4) * lay3.N
            c3["exact"]["quad_kernel_tflops"] = fl3 / (c3["exact"]["phases_ms"]["quad_exact"] * 1e-3) / 1e12
            c3["workload"] = "3D p=4 stiffness, 128^3 elements, sine map, kappa = 1 + 0.5 sin 2pi x1 cos 2pi x2 sin 2pi x3"
            extra["varcoef_3d_p4_128"] = c3
            del b3
        except igs.IGSError as e:
            extra["varcoef_3d_p4_128"] = {"error": str(e)}
        log(f"3D p=4: {extra['varcoef_3d_p4_128']}")

        extra["mesh_dependent_2d_p2_q5"] = mesh_dependent_study(stream)

    # ------------------------------------------------------------ CPU oracle
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(prob, M, q, lay)
        log(f"cpu baseline: {cpu}")

    out = {
        "metric": "assembled nnz/s (surrogate vs quadrature), 3D p=3 128^3; CG+adjoint ms",
        "value": value,
        "unit": "band slots/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3D Poisson stiffness, p=3, 128^3 elements, sine map a=0.05, kappa=1, surrogate M=8 q=3",
                   "dofs": lay.N, "slots": slots, "true_nnz": true_nnz, "parallelism": "single GPU"},
        "true_nnz_per_s": true_nnz / (ms_step * 1e-3),
        "step_ms_separately_timed": step_stats,
        "phases_ms": {k: v["avg_ms"] for k, v in phases.items()},
        "roofline": roofline,
        "step_hbm": step_hbm,
        "rooflines": roofs,
        "cpu_baseline": cpu,
        **extra,
    }
    print(json.dumps(out), flush=True)


def profile_leg(args):
    """Only the timed steps of one leg on the 3D p=3 128^3 workload (M = 8,
    q = 3): the face/edge surrogate assembly (kept plan), or the matrix-free
    apply (its plan executed once, then the products).  Prints one JSON line."""
    import torch

    from paper_1904_06971_amd import igs
    from paper_1904_06971_amd import workloads as W

    prob = W.c4_precision3d()
    lay = igs.layout(prob)
    band = igs.empty_band(prob, torch.float64)
    stream = torch.cuda.current_stream()
    if args.leg in ("face_edge", "per_delta"):
        pl = igs.Plan(prob, igs.STIFFNESS, M=8, q=3, face_edge=args.leg == "face_edge",
                      per_delta=args.leg == "per_delta")
        for _ in range(max(1, args.warmup)):
            pl.execute(out=band)
        ms, ph = timed_plan(pl, band, stream, args.steps)
    else:
        pl = igs.Plan(prob, igs.STIFFNESS, M=8, q=3, matrix_free=True)
        pl.execute(out=band)
        x = torch.as_tensor(W.random_vector(lay.N, 33), device="cuda")
        y = torch.empty_like(x)
        for _ in range(max(1, args.warmup)):
            pl.apply(band, x, dirichlet=True, out=y)
        torch.cuda.synchronize()
        igs.profile_enable(True)
        igs.profile_read()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            pl.apply(band, x, dirichlet=True, out=y)
        e1.record(stream)
        torch.cuda.synchronize()
        pr = igs.profile_read()
        igs.profile_enable(False)
        ms, ph = e0.elapsed_time(e1) / args.steps, {k: v[1] / v[0] for k, v in pr.items()}
    pl.close()
    print(json.dumps({"leg": args.leg, "ms": ms, "phases_ms": ph, "steps": args.steps}), flush=True)


def timed_plan(plan, band, stream, reps):
    """Average step time (HIP events on the launch stream around reps
    back-to-back executions, after one warm execution) and per-phase kernel
    times of a kept plan."""
    import torch

    from paper_1904_06971_amd import igs

    plan.execute(out=band)
    torch.cuda.synchronize()
    igs.profile_enable(True)
    igs.profile_read()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        plan.execute(out=band)
    e1.record(stream)
    torch.cuda.synchronize()
    pr = igs.profile_read()
    igs.profile_enable(False)
    return e0.elapsed_time(e1) / reps, {k: v[1] / v[0] for k, v in pr.items()}


def c2_study(stream, reps):
    """3D Poisson stiffness and mass, p = 3, 64^3 elements on the sine map:
    full quadrature assembly against the surrogate (and its face/edge form) at
    M = 4, 8, 16, q = 3 -- band slots per second, the entry error
    ||A - A~||_max / ||A||_max per M, and the fitted log2 rate of that error
    over M (Thm. RegularityOfStencilFunctions: ~ H^(q+1), slope q+1 = 4)."""
    import torch

    from paper_1904_06971_amd import igs
    from paper_1904_06971_amd import workloads as W

    prob = W.c2_poisson3d()
    lay = igs.layout(prob)
    slots = lay.N * lay.slots
    out = {"workload": "3D Poisson, p=3, 64^3 elements, sine map a=0.05, kappa=1, q=3", "dofs": lay.N, "slots": slots}
    ex = igs.empty_band(prob, torch.float64)
    sb = igs.empty_band(prob, torch.float64)
    for form, fname in ((igs.STIFFNESS, "stiffness"), (igs.MASS, "mass")):
        pe = igs.Plan(prob, form, M=0, q=0)
        ms_ex, _ = timed_plan(pe, ex, stream, reps)
        pe.close()
        scale = float(ex[:, :, :lay.N].abs().max())
        leg = {"exact": {"ms": ms_ex, "slots_per_s": slots / (ms_ex * 1e-3)}}
        for var in ("surrogate", "face_edge", "per_delta"):
            errs = {}
            for M in (4, 8, 16):
                ps = igs.Plan(prob, form, M=M, q=3, face_edge=var == "face_edge", per_delta=var == "per_delta")
                ms_s, ph = timed_plan(ps, sb, stream, reps)
                ps.close()
                err = float((sb[:, :, :lay.N] - ex[:, :, :lay.N]).abs().max()) / scale
                errs[M] = err
                leg["%s_M%d" % (var, M)] = {
                    "ms": ms_s, "slots_per_s": slots / (ms_s * 1e-3), "speedup_vs_exact": ms_ex / ms_s,
                    "rel_max_err": err, "phases_ms": ph}
            leg["rate" if var == "surrogate" else var + "_rate"] = {
                "log2_slope_M4_M8": math.log2(errs[8] / errs[4]), "log2_slope_M8_M16": math.log2(errs[16] / errs[8])}
        out[fname] = leg
    del ex, sb
    return out


def pd_fill_bytes(prob, lay, esize):
    """Algorithmic bytes of the per-delta fill: every entry (i, delta) whose
    row and partner are both cardinal (delta = 0, the diagonal, included),
    written once."""
    n, p = prob["n"], prob["p"]
    C = [lay.m[d] - 2 * p for d in range(n)]
    return math.prod(sum(C[d] - abs(dl) for dl in range(-p, p + 1)) for d in range(n)) * esize


def mesh_dependent_study(stream):
    """The paper's 2D timing study with mesh-dependent sampling lengths
    (Sec. 7.3.3): p = 2, q = 5, M(h) = max{1, floor(c h^((p-q+1/2)/(q+1)))} for
    c in 0.25..4, on the 2D sine map up to about 2.1e6 dofs.  Per mesh: the
    full quadrature assembly and each surrogate assembly, each a kept plan
    timed over 5 executions on the launch stream; speed-up as the paper
    defines it, t_std / t_surr - 1 (in %); the share of rows assembled by
    quadrature (boundary rows plus the sample lattice)."""
    import torch

    from paper_1904_06971_amd import igs
    from paper_1904_06971_amd import workloads as W

    cs = [0.25, 0.5, 0.75, 1.0, 2.0, 3.0, 4.0]
    rows = []

    def timed(pl, band, reps=5):
        pl.execute(out=band)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            pl.execute(out=band)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    for ne in (64, 128, 256, 512, 1024, 1448):
        prob = W.problem(2, 2, ne)
        lay = igs.layout(prob)
        band = igs.empty_band(prob, torch.float64)
        xp = igs.Plan(prob, igs.STIFFNESS, M=0, q=0)
        t_std = timed(xp, band)
        xp.close()
        row = {"nelem": ne, "dofs": lay.N, "std_ms": t_std, "surrogate": {}}
        for c in cs:
            M = igs.sampling_length(ne, 2, 5, c, 0.5)
            st = igs.validate(prob, M, 5)
            if st != 0:
                row["surrogate"][str(c)] = {"M": M, "status": igs.STATUS.get(st, st)}
                continue
            info, _ = igs.surrogate_layout(prob, M, 5)
            sp = igs.Plan(prob, igs.STIFFNESS, M=M, q=5)
            t = timed(sp, band)
            sp.close()
            row["surrogate"][str(c)] = {"M": M, "ms": t, "speedup_pct": (t_std / t - 1) * 100,
                                        "quadrature_rows_pct": 100.0 * info.quadrature_rows / lay.N}
        rows.append(row)
        del band
        log(f"mesh-dependent M, 2D p=2 q=5, nelem {ne}: std {t_std:.3f} ms, " + ", ".join(
            f"c={c}: M={v['M']} " + (f"{v['ms']:.3f} ms" if "ms" in v else v["status"])
            for c, v in row["surrogate"].items()))
    return {"workload": "2D Poisson stiffness, p=2, q=5, sine map a=0.05, kappa=1, M(h) with beta=1/2",
            "rows": rows}


def cpu_model():
    """The host CPU's model name (first /proc/cpuinfo entry), or None."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(prob, M, q, lay):
    """The oracle timed on the host: sample-row quadrature and fit in full, then
    seeded random samples of boundary rows (exact) and analysis-domain rows
    (surrogate), extrapolated to all rows."""
    import numpy as np

    from oracle import oracle as O
    from paper_1904_06971_amd import workloads as W

    O.build()
    m, N, S = O.dims(prob)
    t0 = time.perf_counter()
    sur = O.Surrogate(prob, 0, M, q)
    t_setup = time.perf_counter() - t0
    rows = W.random_rows(N, 60000, 77)
    idx = O.multi_index(prob, rows)
    inner = O.interior_mask(prob, idx)
    rb = rows[~inner][:1500]
    ri = rows[inner][:8000]
    t0 = time.perf_counter()
    O.exact_rows(prob, 0, rb)
    t_b = time.perf_counter() - t0
    t0 = time.perf_counter()
    sur.rows(ri)
    t_i = time.perf_counter() - t0
    nb = N - math.prod(m[d] - 4 * prob["p"] for d in range(3))
    ni = N - nb
    total = t_setup + t_b * nb / len(rb) + t_i * ni / len(ri)
    nthreads = O.threads()
    out = {"value": N * S / total, "unit": "band slots/s", "cores": nthreads, "kind": "oracle",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
           "sample": (f"sample-row quadrature + fit in full ({len(sur.sample_rows)} rows, {t_setup:.1f} s), "
                      f"{len(rb)} random boundary rows ({t_b:.1f} s) and {len(ri)} random analysis-domain rows "
                      f"({t_i:.1f} s), extrapolated to {nb} + {ni} rows: {total:.0f} s for the full band")}
    # the same oracle on one thread (OpenMP of the oracle's C half set to 1):
    # per-row costs of smaller samples, sample rows costed as exact rows
    try:
        import ctypes

        gomp = ctypes.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads(1)
        try:
            rb1, ri1 = rb[:300], ri[:1000]
            t0 = time.perf_counter()
            O.exact_rows(prob, 0, rb1)
            tb1 = (time.perf_counter() - t0) / len(rb1)
            t0 = time.perf_counter()
            sur.rows(ri1)
            ti1 = (time.perf_counter() - t0) / len(ri1)
        finally:
            gomp.omp_set_num_threads(nthreads)
        total1 = tb1 * (nb + len(sur.sample_rows)) + ti1 * ni
        out["single_thread"] = {"value": N * S / total1, "unit": "band slots/s", "cores": 1,
                                "sample": (f"{len(rb1)} boundary rows ({tb1 * 1e3:.2f} ms/row) and {len(ri1)} "
                                           f"analysis-domain rows ({ti1 * 1e3:.3f} ms/row) on one thread, "
                                           f"sample rows costed as boundary rows: {total1:.0f} s for the full band")}
    except OSError:
        pass
    return out


if __name__ == "__main__":
    main()
