"""Benchmark: condensed tangents/s and time-to-1e-8 Newton solve, FP64 vs mixed precision.

Workload: steady lid-driven cavity, 32^3 cells x 6 tets (196,608 tets, 35,937 nodes),
Re 100, Newton to ||R|| <= 1e-8 ||R_0|| (FP64 residual), inexact Newton (Eisenstat-Walker
forcing), GMRES(50) right-preconditioned by 4x4 block-Jacobi (or its learned correction)
with the constant-pressure coarse correction.

value        = condensed tangents/s: n_elems / t(vms_condense_assemble), the median of 20
               calls after 3 warm-ups, each call bracketed by HIP events on its stream
               (element residual + tangent + FP64 K_ff^-1 + Schur condensation + scatter into
               4x4 block-CSR + Dirichlet elimination + residual norm), mixed precision,
               at the workload's initial state; cpu_baseline measures the same on the oracle.
ms_per_step  = time to 1e-8 of the headline form (mixed + learned correction, GMRES restarts
               deflated by DEFLATE harmonic Ritz vectors): one step is a
               complete Newton-Schur solve from the initial state (every assembly,
               preconditioner setup, GMRES iteration, recovery and residual evaluation), all on
               the GPU through the C ABI, inputs resident on the device before the timed region.
The learned correction is trained and selected on Newton systems of other Reynolds numbers
(cavity 32^3 at Re 75 and 125); the timed Re 100 solve is never seen in training.
Also reported: every form's time to 1e-8, the assembly and Arnoldi-SpMV rooflines (HIP events on
the launch stream), the 64^3 jittered cube (the HBM-resident size) and the CPU oracle.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6      # vector FP64
FP32_PEAK_TFLOPS = 78.6      # vector FP32 without packed instructions (packed FP32 is not used)
PROFILE_EVERY = 8            # timed region: HIP events on the dominant kernel's launches in every 8th GMRES cycle
COUNTER_ITERS = 64           # --counters: Arnoldi steps (SpMV launches) in the counter run
COPY_MIB = 256               # --counters: size of the reference copy
KERNEL_OF_PHASE = {"condense": "tile_kernel", "spmv": "spmv_kernel", "dots": "dots_kernel",
                   "update": "update_fused_kernel", "pc_apply": "ap_blocks_kernel"}
TRAIN_RE = (75.0, 125.0)     # Reynolds numbers of the learned correction's training systems
DEFLATE = 10                 # harmonic Ritz vectors kept by the deflated-restart forms (GMRES(50))
WORKLOAD_TEXT = ("lid-driven cavity 32^3 cells x 6 tets ({ne} tets, {nn} nodes), Re {re:g}, steady Newton to "
                 "1e-8 with Eisenstat-Walker forcing, GMRES(50) right-preconditioned by 4x4 block-Jacobi "
                 "(learned correction in the headline form) plus the constant-pressure coarse correction; "
                 "value = n_elems / t(vms_condense_assemble), mixed; ms_per_step = time to 1e-8, "
                 "mixed + learned, deflated restarts (10 harmonic Ritz vectors kept)")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cavity32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-hbm-config", action="store_true", help="skip the 64^3 jittered-cube measurements")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="elements in the oracle sample (0: every element of the workload)")
    ap.add_argument("--study", choices=["bfs", "nr", "picard", "jet", "es"], default=None,
                    help="bfs: the learned-correction study on the backward-facing step (train on the steady "
                         "Re 400..800 continuation of bfs8, compare block-Jacobi FP64, block-Jacobi mixed and "
                         "the learned correction over the transient bfs16 run); prints its own JSON report "
                         "instead of the bench line")
    ap.add_argument("--study-steps", type=int, default=2,
                    help="time steps of the transient run in --study bfs (bfs16) and --study jet (jet8)")
    ap.add_argument("--study-restart", type=int, default=50,
                    help="GMRES restart length of the bfs16 evaluation in --study bfs")
    ap.add_argument("--study-forms", default="fp64_bj,mixed_bj,mixed_learned,fp64_dr,mixed_b64_dr",
                    help="comma-separated forms of the bfs16 evaluation in --study bfs")
    ap.add_argument("--counters", action="store_true",
                    help="short run for hardware-counter passes: one condensed assembly and GMRES on the "
                         "workload's mixed-precision tangent capped at COUNTER_ITERS Arnoldi steps, then a "
                         "COPY_MIB device-to-device copy (the scale reference for the counters)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def event_median_us(fn, reps=20, warm=3):
    """Median duration of fn() over reps calls, each bracketed by HIP events on the current stream."""
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    ts = sorted(a.elapsed_time(b) * 1e3 for a, b in ev)
    return ts[len(ts) // 2]


def assembly_bench(B, ctx, mesh, u, beta, re, dt=0.0, u_prev=None):
    """n_elems / t(vms_condense_assemble) (median of 20 event-timed calls after 3 warm-ups) and
    the tile kernel's own time and algorithmic bytes from the phase timers."""
    import torch
    A = ctx.new_bsr()
    rhs = ctx.new_vec()
    rn = torch.zeros(1, dtype=torch.float64, device=ctx.device)

    def call():
        B.vms_condense_assemble(ctx, u, beta, re, dt, u_prev, None, A, rhs, rn)

    t_us = event_median_us(call)
    B.vms_profile(ctx, True, phases=["condense"])
    for _ in range(20):
        call()
    ms, cnt, byt = B.vms_profile_read(ctx)["condense"]
    B.vms_profile(ctx, False)
    kern_us = 1e3 * ms / cnt
    return {"tangents_per_s": mesh.n_elems / (t_us * 1e-6), "call_us": t_us, "kernel_us": kern_us,
            "alg_bytes_per_launch": byt / cnt, "alg_GBps": byt / cnt / (kern_us * 1e-6) / 1e9}


# Algorithmic flops of one element's condensed tangent and residual (closed-form element,
# backward Euler, no body force), counted term by term from the tile kernel's formulas with
# every quantity the element's four rows share counted once (add, sub, mul, div = 1 flop):
#   FP64, per element: geometry 87, fields 128, R_f 84, K_ff and its inverse 78;
#         per row vertex: R_c 121, K_cf 65, K_ff^-1 R_f and R* 39, Y = K_cf K_ff^-1 60
#   precision T, per row vertex: block factors 165; per (row, column) block 111
ELEM_FLOPS_FP64 = 87 + 128 + 84 + 78 + 4 * (121 + 65 + 39 + 60)
ELEM_FLOPS_T = 4 * (165 + 4 * 111)


def assembly_roofline(res, n_elems, mixed, workload):
    """HBM and VALU fractions of the tile kernel; traffic from the committed counter summary
    (taken on the mixed-precision kernel, so null for FP64)."""
    alg = res["alg_bytes_per_launch"]
    t = res["kernel_us"] * 1e-6
    f64 = ELEM_FLOPS_FP64 * n_elems
    ft = ELEM_FLOPS_T * n_elems
    # both precisions run at the same vector rate here (FP32 without packed instructions)
    valu_frac = (f64 + ft) / t / 1e12 / FP64_PEAK_TFLOPS
    traffic, traffic_src = measured_traffic(workload, "condense") if mixed else (None, None)
    return {"bound": "hbm", "kernel": "tile_kernel", "achieved": round(alg / t / 1e9, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(alg / t / 1e9 / HBM_PEAK_GBS, 4), "alg_bytes_per_launch": alg,
            "avg_launch_us": round(res["kernel_us"], 3), "traffic": traffic, "traffic_source": traffic_src,
            "alu": {"flops_per_elem_fp64": ELEM_FLOPS_FP64, "flops_per_elem_" + ("fp32" if mixed else "fp64_blocks"):
                    ELEM_FLOPS_T, "achieved_tflops": round((f64 + ft) / t / 1e12, 2),
                    "peak_tflops": FP64_PEAK_TFLOPS, "frac": round(valu_frac, 4)}}


def cache_probe_gbps(nbytes):
    """Bandwidth a working set of nbytes sees when it is reused back to back (so that it stays
    in the L2 and Infinity Cache): a device-to-device copy that reads nbytes / 2 and writes
    nbytes / 2, median of 20 after 5 warm-ups, HIP events.  (A float32 sum over the same bytes
    reached 1.8 TB/s at 37 MB, less than the SpMV itself; the copy 4.5 TB/s.)"""
    import torch
    n = max(1, nbytes // 8)
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    t_us = event_median_us(lambda: dst.copy_(src), reps=20, warm=5)
    return 2 * n * 4 / (t_us * 1e-6) / 1e9


def spmv_roofline(prof, phase):
    ms, cnt, byt = prof[phase]
    achieved = byt / cnt / (ms / cnt / 1e3) / 1e9
    return {"bound": "hbm", "kernel": KERNEL_OF_PHASE.get(phase, phase), "phase": phase,
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "avg_launch_us": round(1e3 * ms / cnt, 3),
            "launches_timed": cnt, "timed_every": PROFILE_EVERY, "alg_bytes_per_launch": byt / cnt}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU path is not built.",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_0809_4802_amd import binding as B, driver, learned
    from workloads import build_workload

    dev = "cuda:0"
    if args.study == "bfs":
        bfs_study(B, driver, learned, build_workload, dev, args.study_steps, args.study_restart,
                  args.study_forms.split(","))
        return
    if args.study == "nr":
        nr_study(B, driver, build_workload, dev, args.workload)
        return
    if args.study == "picard":
        picard_study(B, driver, build_workload, dev, args.workload)
        return
    if args.study == "jet":
        jet_study(B, driver, build_workload, dev, args.study_steps)
        return
    if args.study == "es":
        es_study(B, driver, build_workload, dev)
        return
    cfg, mesh, u0, beta0, bc = build_workload(args.workload)
    if args.counters:
        counter_run(B, cfg, mesh, u0, beta0, bc, dev)
        return
    xyz = torch.from_numpy(mesh.xyz).to(dev)
    tets = torch.from_numpy(mesh.tets).to(dev)
    dd = torch.from_numpy(bc.dofs).to(dev)
    u0d = torch.from_numpy(u0).to(dev)
    b0d = torch.from_numpy(beta0).to(dev)
    log(f"workload {args.workload}: {mesh.n_elems} tets, {mesh.n_nodes} nodes, Re {cfg.re}")

    def lin_opts(weights=None, deflate=0, b64=0):
        return B.solve_opts(restart=50, rtol=1e-9, max_iters=60000,
                            pc=B.VMS_PC_LEARNED if weights is not None else B.VMS_PC_BLOCK_JACOBI,
                            pc_weights=weights, deflate=deflate, basis_fp64=b64)

    def solve(ctx, weights=None, re=cfg.re, deflate=0, b64=0):
        u = u0d.clone()
        beta = b0d.clone()
        torch.cuda.synchronize()
        return driver.newton_solve(ctx, u, beta, re, tol=cfg.newton_tol, lin=lin_opts(weights, deflate, b64),
                                   forcing="ew", max_newton=30)

    ctxs = {"fp64": B.Context(xyz, tets, dd, precision=B.VMS_FP64),
            "mixed": B.Context(xyz, tets, dd, precision=B.VMS_MIXED)}
    headline = "mixed"
    headline_form = "mixed_learned_dr"     # the timed solves: mixed + learned + deflated restarts

    # ---- metric 1: condensed tangents/s = n_elems / t(vms_condense_assemble)
    assembly = {}
    for name, ctx in ctxs.items():
        assembly[name] = assembly_bench(B, ctx, mesh, u0d, b0d, cfg.re)
        assembly[name]["roofline"] = assembly_roofline(assembly[name], mesh.n_elems, name == "mixed", args.workload)
        log(f"assembly {name}: {assembly[name]}")

    # ---- the solves run on deterministic contexts (one-wavefront assembly tiles): the
    # assemblies, and with them the GMRES iteration counts, the learned training data and the
    # selected weights, are bitwise reproducible from run to run; the assembly is about 1.3x
    # slower there, under 0.3% of a solve
    for c in ctxs.values():
        c.close()
    ctxs = {"fp64": B.Context(xyz, tets, dd, precision=B.VMS_FP64, deterministic=True),
            "mixed": B.Context(xyz, tets, dd, precision=B.VMS_MIXED, deterministic=True, basis_fp64=True)}

    # ---- learned block-Jacobi correction, held out: trained on the method's own condensed
    # tangents and GMRES restart residuals from mixed-precision Newton solves of this mesh at
    # other Reynolds numbers; checkpoints are scored by GMRES iterations on the last Newton
    # system of each training solve, which are held out of the training batches
    t0 = time.perf_counter()
    ctx = ctxs["mixed"]
    train, val = [], []
    for re in TRAIN_RE:
        d, _ = learned.collect_newton_data(ctx, u0d.clone(), b0d.clone(), re,
                                           lin=B.solve_opts(restart=50, rtol=1e-4, max_iters=60000), per_step=48)
        train += d[:-1]
        val.append((d[-1][0], d[-1][1][0].contiguous()))
    weights, train_report = learned.train_select(ctx, train or [v for v in val], val, seeds=(1, 2, 3), steps=300,
                                                 lr=3e-4, lr_decay="cosine", check_every=10)
    train_report["seconds"] = time.perf_counter() - t0
    train_report["training_systems"] = (f"cavity32 mixed Newton solves at Re {', '.join(f'{r:g}' for r in TRAIN_RE)}: "
                                        f"{len(train)} systems for training, the last system of each solve "
                                        f"({len(val)}) for checkpoint selection; the timed Re {cfg.re:g} solve "
                                        f"is not among them")
    log(f"learned PC: { {k: v for k, v in train_report.items() if k != 'runs'} }")
    del train, val

    # ---- metric 2: time to 1e-8 in every form (one warm-up + one timed solve each); the _dr
    # forms restart GMRES with deflation
    forms = {}
    for name, ctx_name, w, defl, b64 in (("fp64_bj", "fp64", None, 0, 0), ("mixed_bj", "mixed", None, 0, 0),
                                         ("mixed_learned", "mixed", weights, 0, 0),
                                         ("fp64_bj_dr", "fp64", None, DEFLATE, 0),
                                         ("mixed_bj_dr", "mixed", None, DEFLATE, 0),
                                         ("mixed_learned_dr", "mixed", weights, DEFLATE, 0),
                                         ("mixed_b64_dr", "mixed", None, DEFLATE, 1),
                                         ("mixed_learned_b64_dr", "mixed", weights, DEFLATE, 1)):
        if name.startswith("mixed_learned") and w is None:
            plain = name.replace("mixed_learned", "mixed_bj" if not b64 else "mixed")
            forms[name] = dict(forms[plain], note="validation selected plain block-Jacobi")
            continue
        solve(ctxs[ctx_name], w, deflate=defl, b64=b64)
        r = solve(ctxs[ctx_name], w, deflate=defl, b64=b64)
        forms[name] = {"seconds": r.seconds, "newton_steps": len(r.rnorms) - 1,
                       "gmres_iters": int(sum(d["iters"] for d in r.lin)),
                       # GMRES cycles (inner FP32 cycles in the mixed form); a cycle replayed
                       # from its graph launches all `restart` steps, those after convergence
                       # return at once
                       "gmres_cycles": int(sum(d["restarts"] for d in r.lin)),
                       "fell_back_to_bj": int(sum(d["fell_back_to_bj"] for d in r.lin)),
                       "deflation_stopped": int(sum(d["deflation_stopped"] for d in r.lin)),
                       "final_rel_residual": r.rnorms[-1] / r.rnorms[0]}
        log(f"time-to-1e-8 {name}: {forms[name]}")

    # ---- phase breakdown of one headline solve, every phase timed (outside the timed region)
    ctx = ctxs[headline]
    B.vms_profile(ctx, True)
    solve(ctx, weights, deflate=DEFLATE)
    prof_all = B.vms_profile_read(ctx)
    B.vms_profile(ctx, False)
    phases = {p: {"ms": round(v[0], 3), "launches": v[1], "avg_us": round(1e3 * v[0] / v[1], 3) if v[1] else None,
                  "alg_GBps": round(v[2] / v[0] / 1e6, 1) if v[0] else None} for p, v in prof_all.items() if v[1]}
    # the roofline kernel: the Arnoldi SpMV, the kernel with the most GPU time per solve in the
    # kernel trace (about 30%, the update 28%, the dots 20%); the event-timed breakdown above
    # brackets every launch and inflates the short update and dots launches more
    phase = "spmv"

    # ---- timed region: K headline solves (mixed precision + learned correction + deflated
    # restarts); only the
    # dominant kernel's launches carry HIP events (on the stream they are launched on)
    for _ in range(args.warmup):
        solve(ctx, weights, deflate=DEFLATE)
    B.vms_profile(ctx, True, phases=[phase], every=PROFILE_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = []
    for _ in range(args.steps):
        steps.append(solve(ctx, weights, deflate=DEFLATE))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = B.vms_profile_read(ctx)
    B.vms_profile(ctx, False)

    roofline = spmv_roofline(prof, phase)
    traffic, traffic_src = measured_traffic(args.workload, phase)
    roofline["traffic"] = traffic
    roofline["traffic_source"] = traffic_src
    # the 37 MB matrix of this size stays in the 256 MB Infinity Cache between launches: its
    # bandwidth is also given against a copy of the same working set
    probe = cache_probe_gbps(int(roofline["alg_bytes_per_launch"]))
    roofline["cache_probe_GBps"] = round(probe, 1)
    roofline["frac_vs_cache_probe"] = round(roofline["achieved"] / probe, 4)
    log(f"roofline: {roofline}")
    for c in ctxs.values():
        c.close()
    del ctxs
    torch.cuda.empty_cache()

    # ---- the 64^3 jittered cube: matrix and basis far beyond the caches
    hbm = None
    if not args.no_hbm_config:
        hbm = hbm_config(B, build_workload, dev)

    # ---- CPU oracle baseline on a bounded sample of the same workload
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(mesh, u0, beta0, bc, cfg, args.cpu_sample, forms)

    out = {
        "metric": "condensed tangents/s + time-to-1e-8 Newton step, plain FP64 vs mixed+learned-PC",
        "value": assembly[headline]["tangents_per_s"],
        "unit": "condensed tangents/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if headline == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: " + WORKLOAD_TEXT.format(ne=mesh.n_elems, nn=mesh.n_nodes,
                                                                          re=cfg.re),
                   "n_elems": mesh.n_elems, "n_nodes": mesh.n_nodes},
        "time_to_1e-8_s": {k: v["seconds"] for k, v in forms.items()},
        "mixed_learned_speedup_vs_fp64_bj": forms["fp64_bj"]["seconds"] / forms["mixed_learned"]["seconds"],
        "headline_form": headline_form,
        "headline_speedup_vs_fp64_bj": forms["fp64_bj"]["seconds"] / forms[headline_form]["seconds"],
        "forms": forms,
        "learned_pc": train_report,
        "deterministic_solves": True,
        "assembly": assembly,
        "phases": phases,
        "roofline": roofline,
        "hbm_config": hbm,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def hbm_config(B, build_workload, dev, gmres_steps=150):
    """es64 (64^3 jittered cube, 1,572,864 tets, first backward-Euler step of the Ethier-Steinman
    flow): condensed assembly (FP64, mixed) and the Arnoldi SpMV (mixed, the first
    gmres_steps Arnoldi steps of GMRES(50) on the mixed tangent, every launch event-timed)."""
    import torch
    cfg, mesh, u0, beta0, bc = build_workload("es64")
    xyz = torch.from_numpy(mesh.xyz).to(dev)
    tets = torch.from_numpy(mesh.tets).to(dev)
    dd = torch.from_numpy(bc.dofs).to(dev)
    u = torch.from_numpy(u0).to(dev)
    b = torch.from_numpy(beta0).to(dev)
    out = {"workload": f"es64: {mesh.n_elems} tets, {mesh.n_nodes} nodes, Re {cfg.re:g}, dt {cfg.dt:g}"}
    for name, prec in (("fp64", B.VMS_FP64), ("mixed", B.VMS_MIXED)):
        ctx = B.Context(xyz, tets, dd, precision=prec)
        res = assembly_bench(B, ctx, mesh, u, b, cfg.re, cfg.dt, u)
        res["roofline"] = assembly_roofline(res, mesh.n_elems, name == "mixed", "es64")
        out[f"assembly_{name}"] = res
        log(f"es64 assembly {name}: {res}")
        if name == "mixed":
            A, rhs, _ = B.vms_condense_assemble(ctx, u, b, cfg.re, cfg.dt, u)
            x = ctx.new_vec()
            B.vms_profile(ctx, True, phases=["spmv", "dots", "update"], every=1)
            B.vms_gmres_solve(ctx, A, rhs, x, B.solve_opts(restart=50, rtol=1e-14, max_iters=gmres_steps),
                              allow_noconv=True)
            prof = B.vms_profile_read(ctx)
            B.vms_profile(ctx, False)
            out["spmv_mixed"] = spmv_roofline(prof, "spmv")
            out["spmv_mixed"]["timed_every"] = 1
            out["spmv_mixed"]["traffic"], out["spmv_mixed"]["traffic_source"] = measured_traffic("es64", "spmv")
            for p in ("dots", "update"):
                ms, cnt, byt = prof[p]
                out[f"{p}_mixed"] = {"avg_launch_us": round(1e3 * ms / cnt, 3),
                                     "alg_GBps": round(byt / ms / 1e6, 1), "launches": cnt}
            log(f"es64 spmv: {out['spmv_mixed']}")
            del A, rhs, x
        ctx.close()
        torch.cuda.empty_cache()
    return out


def nr_study(B, driver, build_workload, dev, workload):
    """Newton-Raphson on the uncondensed system (coarse and fine unknowns together, Section 4.2)
    against Newton-Schur (Section 5), time to 1e-8 from the same initial state, FP64 and
    mixed precision, GMRES(50) with inexact-Newton forcing in both.  Newton-Raphson is
    preconditioned by block-Jacobi with the Schur complement's diagonal blocks on node rows and
    K_ff^-1 on element rows, plus the constant-pressure coarse correction."""
    import torch
    cfg, mesh, u0, beta0, bc = build_workload(workload)
    xyz = torch.from_numpy(mesh.xyz).to(dev)
    tets = torch.from_numpy(mesh.tets).to(dev)
    dd = torch.from_numpy(bc.dofs).to(dev)
    u0d = torch.from_numpy(u0).to(dev)
    b0d = torch.from_numpy(beta0).to(dev)
    report = {"study": "nr", "workload": workload, "n_elems": mesh.n_elems, "n_nodes": mesh.n_nodes,
              "unknowns": {"schur": 4 * mesh.n_nodes, "full": 4 * mesh.n_nodes + 3 * mesh.n_elems}}
    for prec_name, prec in (("fp64", B.VMS_FP64), ("mixed", B.VMS_MIXED)):
        ctx = B.Context(xyz, tets, dd, precision=prec, full_system=True)
        for method in ("schur", "full"):
            runs = []
            for _ in range(2):                     # warm, timed
                u = u0d.clone()
                beta = b0d.clone()
                torch.cuda.synchronize()
                runs.append(driver.newton_solve(ctx, u, beta, cfg.re, tol=cfg.newton_tol,
                                                lin=B.solve_opts(restart=50, rtol=1e-9, max_iters=60000),
                                                forcing="ew", max_newton=30, method=method))
            r = runs[-1]
            key = f"{prec_name}_{method}"
            report[key] = {"seconds": r.seconds, "newton_steps": len(r.rnorms) - 1,
                           "gmres_iters": int(sum(d["iters"] for d in r.lin)),
                           "gmres_iters_per_step": [int(d["iters"]) for d in r.lin],
                           "final_rel_residual": r.rnorms[-1] / r.rnorms[0]}
            log(f"{key}: {report[key]}")
        report[f"{prec_name}_schur_speedup"] = report[f"{prec_name}_full"]["seconds"] / report[f"{prec_name}_schur"]["seconds"]
        del ctx
    print(json.dumps(report), flush=True)


def picard_study(B, driver, build_workload, dev, workload, reynolds=(100.0, 400.0, 1000.0), max_steps=60):
    """Consistent Newton (Section 4.2) against the fixed-point linearisation the introduction
    argues against (advecting velocity held at the iterate), mixed precision, from the same
    initial state, to 1e-8 or max_steps, inexact-Newton forcing and GMRES(50) in both."""
    import torch
    cfg, mesh, u0, beta0, bc = build_workload(workload)
    ctx = B.Context(torch.from_numpy(mesh.xyz).to(dev), torch.from_numpy(mesh.tets).to(dev),
                    torch.from_numpy(bc.dofs).to(dev), precision=B.VMS_MIXED)
    report = {"study": "picard", "workload": workload, "n_elems": mesh.n_elems}
    for re in reynolds:
        for name, kind in (("newton", B.VMS_LIN_NEWTON), ("picard", B.VMS_LIN_PICARD)):
            B.vms_set_linearization(ctx, kind)
            u = torch.from_numpy(u0).to(dev)
            beta = torch.from_numpy(beta0).to(dev)
            try:
                r = driver.newton_solve(ctx, u, beta, re, tol=cfg.newton_tol,
                                        lin=B.solve_opts(restart=50, rtol=1e-9, max_iters=60000),
                                        forcing="ew", max_newton=max_steps, raise_on_fail=False)
                out = {"converged": bool(r.converged), "steps": len(r.rnorms) - 1, "seconds": r.seconds,
                       "gmres_iters": int(sum(d["iters"] for d in r.lin)),
                       "rel_residuals": [x / r.rnorms[0] for x in r.rnorms]}
            except B.VmsError as e:          # a linear solve that fails is a result here
                out = {"converged": False, "error": str(e)}
            key = f"re{re:g}_{name}"
            report[key] = out
            log(f"{key}: " + json.dumps({k: v for k, v in out.items() if k != "rel_residuals"}))
    B.vms_set_linearization(ctx, B.VMS_LIN_NEWTON)
    print(json.dumps(report), flush=True)


def jet_study(B, driver, build_workload, dev, steps):
    """The jet from an orifice (jet8: 196,608 tets, Re 1000, backward Euler dt 0.01 from rest):
    `steps` time steps in each precision, Newton to 1e-8 per step with GMRES(50) + block-Jacobi;
    per step the Newton iterations, GMRES iterations, seconds and the largest velocity."""
    import numpy as np
    import torch
    cfg, mesh, u0, beta0, bc = build_workload("jet8")
    dofs = torch.from_numpy(bc.dofs.astype(np.int64)).to(dev)
    vals = torch.from_numpy(bc.values).to(dev)
    report = {"study": "jet", "workload": "jet8", "n_elems": mesh.n_elems, "re": cfg.re, "dt": cfg.dt,
              "steps": steps}
    for name, prec in (("fp64_bj", B.VMS_FP64), ("mixed_bj", B.VMS_MIXED)):
        ctx = B.Context(torch.from_numpy(mesh.xyz).to(dev), torch.from_numpy(mesh.tets).to(dev),
                        torch.from_numpy(bc.dofs).to(dev), precision=prec)
        u = torch.from_numpy(u0).to(dev)
        beta = torch.from_numpy(beta0).to(dev)
        u_prev = torch.empty_like(u)
        per_step = []
        for _ in range(steps):
            u_prev.copy_(u)
            driver.set_dirichlet(u, dofs, vals)
            r = driver.newton_solve(ctx, u, beta, cfg.re, cfg.dt, u_prev, None, tol=cfg.newton_tol,
                                    lin=B.solve_opts(restart=50, rtol=1e-9, max_iters=40000))
            per_step.append({"newton": len(r.rnorms) - 1, "gmres_iters": int(sum(d["iters"] for d in r.lin)),
                             "seconds": r.seconds, "max_speed": float(u[:, :3].norm(dim=1).max())})
        report[name] = {"seconds": sum(p["seconds"] for p in per_step),
                        "gmres_iters": sum(p["gmres_iters"] for p in per_step), "per_step": per_step}
        log(f"jet {name}: {report[name]['seconds']:.3f} s, {report[name]['gmres_iters']} GMRES iterations")
        ctx.close()
    print(json.dumps(report), flush=True)


def es_study(B, driver, build_workload, dev, forms=("fp64_bj", "mixed_bj", "fp64_dr", "mixed_dr", "mixed_b64_dr")):
    """The Ethier-Steinman transient of config 3 (es64: 64^3 jittered cube, 1,572,864 tets,
    Re 1000, backward Euler dt 0.01, 10 steps, the exact boundary values at every t_{n+1}): per
    form the Newton steps (to 1e-8, Eisenstat-Walker forcing), GMRES(50) iterations and seconds
    of every time step.  Forms as in the bfs study: fp64 / mixed precision, _dr with deflated
    restarts (DEFLATE kept), b64 with an FP64 basis on the mixed context."""
    import numpy as np
    import torch
    from workloads import ethier_steinman_bc
    cfg, mesh, u0, beta0, bc = build_workload("es64")
    nu_l = 2.0 / cfg.re
    dofs = torch.from_numpy(bc.dofs.astype(np.int64)).to(dev)
    report = {"study": "es", "workload": "es64", "n_elems": mesh.n_elems, "n_nodes": mesh.n_nodes, "re": cfg.re,
              "dt": cfg.dt, "steps": cfg.steps, "restart": 50}
    values = [torch.from_numpy(ethier_steinman_bc(mesh, (n + 1) * cfg.dt, nu_l).values).to(dev)
              for n in range(cfg.steps)]
    for name in forms:
        prec = B.VMS_FP64 if name.startswith("fp64") else B.VMS_MIXED
        defl = DEFLATE if name.endswith("_dr") else 0
        b64 = 1 if "_b64" in name else 0
        ctx = B.Context(torch.from_numpy(mesh.xyz).to(dev), torch.from_numpy(mesh.tets).to(dev),
                        torch.from_numpy(bc.dofs).to(dev), precision=prec, basis_fp64=bool(b64))
        u = torch.from_numpy(u0).to(dev)
        beta = torch.from_numpy(beta0).to(dev)
        u_prev = torch.empty_like(u)
        per_step = []
        for n in range(cfg.steps):
            u_prev.copy_(u)
            driver.set_dirichlet(u, dofs, values[n])
            r = driver.newton_solve(ctx, u, beta, cfg.re, cfg.dt, u_prev, None, tol=cfg.newton_tol, forcing="ew",
                                    lin=B.solve_opts(restart=50, rtol=1e-9, max_iters=400000, deflate=defl,
                                                     basis_fp64=b64))
            per_step.append({"newton": len(r.rnorms) - 1, "gmres_iters": int(sum(d["iters"] for d in r.lin)),
                             "seconds": r.seconds,
                             "deflation_stopped": int(sum(d["deflation_stopped"] for d in r.lin))})
        report[name] = {"seconds": sum(p["seconds"] for p in per_step),
                        "newton_steps": sum(p["newton"] for p in per_step),
                        "gmres_iters": sum(p["gmres_iters"] for p in per_step), "per_step": per_step}
        log(f"es64 {name}: {report[name]['seconds']:.3f} s, {report[name]['newton_steps']} Newton steps, "
            f"{report[name]['gmres_iters']} GMRES iterations")
        ctx.close()
        torch.cuda.empty_cache()
    print(json.dumps(report), flush=True)


def bfs_study(B, driver, learned, build_workload, dev, steps, restart=50, forms=("fp64_bj", "mixed_bj", "mixed_learned")):
    """Learned correction on the backward-facing step.  Training data: the Newton systems of the
    steady bfs8 continuation Re 400 -> 800 and of the first backward-Euler steps of bfs8 at
    Re 800, dt 0.05 from an impulsive start (mixed, GMRES(50) + block-Jacobi, restart residuals
    logged); the last two transient systems are held out for checkpoint selection.  Evaluation: the
    transient bfs16 run (Re 800, dt 0.05, impulsive start) for `steps` steps in each form --
    FP64 + block-Jacobi, mixed + block-Jacobi, mixed + learned correction -- Newton to 1e-8 per
    step, GMRES(restart); Newton steps, GMRES iterations and wall time per step."""
    import numpy as np
    import torch
    report = {"study": "bfs", "forms": list(forms)}
    weights = None
    if any(f.startswith("mixed_learned") for f in forms):
        t0 = time.perf_counter()
        cfg8, m8, u8, b8, bc8 = build_workload("bfs8")
        ctx8 = B.Context(torch.from_numpy(m8.xyz).to(dev), torch.from_numpy(m8.tets).to(dev),
                         torch.from_numpy(bc8.dofs).to(dev), precision=B.VMS_MIXED, max_restart=max(50, restart))
        lin8 = B.solve_opts(restart=50, rtol=1e-4, max_iters=20000)
        u = torch.from_numpy(u8).to(dev)
        beta = torch.from_numpy(b8).to(dev)
        data, cont = [], []
        for re in cfg8.re_sweep:
            tr = time.perf_counter()
            d, hist = learned.collect_newton_data(ctx8, u, beta, re, tol=cfg8.newton_tol, max_newton=12, lin=lin8,
                                                  per_step=32, allow_noconv=True)
            converged = hist[-1] <= cfg8.newton_tol * hist[0]
            cont.append({"re": re, "newton_steps": len(d), "converged": bool(converged),
                         "seconds": round(time.perf_counter() - tr, 2),
                         "rnorms": [float(f"{r:.3e}") for r in hist]})
            log(f"bfs8 steady Re {re:g}: {cont[-1]}")
            data += d
            if not converged:
                break
        # transient bfs8 systems, impulsive start
        u = torch.from_numpy(u8).to(dev)
        beta = torch.from_numpy(b8).to(dev)
        u_prev = torch.empty_like(u)
        trans = []
        for n in range(2):
            tr = time.perf_counter()
            u_prev.copy_(u)
            d, hist = learned.collect_newton_data(ctx8, u, beta, 800.0, 0.05, u_prev, tol=1e-8, max_newton=8,
                                                  lin=lin8, per_step=32, allow_noconv=True)
            trans += d
            log(f"bfs8 transient step {n}: Newton {len(d)}, {time.perf_counter() - tr:.1f} s")
        report["bfs8"] = {"n_elems": m8.n_elems, "n_nodes": m8.n_nodes, "continuation": cont,
                          "transient_systems": len(trans), "training_systems": len(data) + len(trans) - 2,
                          "seconds": time.perf_counter() - t0}
        t1 = time.perf_counter()
        # the last two transient systems are held out for checkpoint selection
        train_set = data + trans[:-2]
        val = [(A, S[0].contiguous()) for A, S in trans[-2:]]
        weights, train = learned.train_validated(ctx8, train_set, val, steps=300, lr=3e-4, check_every=25,
                                                 val_restart=restart, val_max_iters=60000)
        train["seconds"] = time.perf_counter() - t1
        report["training"] = train
        log(f"training: {train}")
        del data, trans, train_set, val
        ctx8.close()
        torch.cuda.empty_cache()

    cfg, m, u0, beta0, bc = build_workload("bfs16")
    dofs = torch.from_numpy(bc.dofs.astype(np.int64)).to(dev)
    vals = torch.from_numpy(bc.values).to(dev)
    report["bfs16"] = {"n_elems": m.n_elems, "n_nodes": m.n_nodes, "re": cfg.re, "dt": cfg.dt, "steps": steps,
                       "restart": restart}
    for name in forms:
        prec = B.VMS_FP64 if name.startswith("fp64") else B.VMS_MIXED
        # a form ending in _dr restarts GMRES with deflation (DEFLATE harmonic Ritz vectors kept);
        # one with b64 runs a mixed context's GMRES on an FP64 basis
        defl = DEFLATE if name.endswith("_dr") else 0
        b64 = 1 if "_b64" in name else 0
        w = weights if name.startswith("mixed_learned") else None
        if name.startswith("mixed_learned") and w is None:
            report["bfs16"][name] = "validation selected plain block-Jacobi"
            continue
        ctx = B.Context(torch.from_numpy(m.xyz).to(dev), torch.from_numpy(m.tets).to(dev),
                        torch.from_numpy(bc.dofs).to(dev), precision=prec, max_restart=max(50, restart),
                        basis_fp64=bool(b64))
        u = torch.from_numpy(u0).to(dev)
        beta = torch.from_numpy(beta0).to(dev)
        u_prev = torch.empty_like(u)
        per_step = []
        for n in range(steps):
            u_prev.copy_(u)
            driver.set_dirichlet(u, dofs, vals)
            lin = B.solve_opts(restart=restart, rtol=1e-9, max_iters=400000,
                               pc=B.VMS_PC_LEARNED if w is not None else B.VMS_PC_BLOCK_JACOBI, pc_weights=w,
                               deflate=defl, basis_fp64=b64)
            r = driver.newton_solve(ctx, u, beta, cfg.re, cfg.dt, u_prev, None, tol=cfg.newton_tol, lin=lin,
                                    forcing="ew")
            per_step.append({"seconds": r.seconds, "newton": len(r.rnorms) - 1,
                             "gmres": int(sum(d["iters"] for d in r.lin)),
                             "fell_back": int(sum(d["fell_back_to_bj"] for d in r.lin)),
                             "deflation_stopped": int(sum(d["deflation_stopped"] for d in r.lin)),
                             "rel_residual": r.rnorms[-1] / r.rnorms[0]})
            log(f"bfs16 {name} step {n}: {per_step[-1]}")
        secs = [p["seconds"] for p in per_step]
        report["bfs16"][name] = {
            "gmres_iters": int(sum(p["gmres"] for p in per_step)),
            "newton_steps": int(sum(p["newton"] for p in per_step)),
            "seconds": float(sum(secs)), "seconds_per_step_mean": float(np.mean(secs)),
            "seconds_per_step_max": float(np.max(secs)),
            "fell_back_to_bj": int(sum(p["fell_back"] for p in per_step)),
            "per_step": per_step}
        log(f"bfs16 {name}: " + json.dumps({k: v for k, v in report["bfs16"][name].items() if k != "per_step"}))
        ctx.close()
        torch.cuda.empty_cache()
    print(json.dumps(report), flush=True)


def spmv_source_hash():
    """sha256 of the SpMV section of the GMRES source (the kernel the counters were taken on)."""
    import hashlib
    src = open(os.path.join(ROOT, "paper_0809_4802_amd", "csrc", "krylov.hip")).read()
    a = src.index("// " + "-" * 82 + " SpMV")
    b = src.index("// " + "-" * 75 + " block-Jacobi")
    return hashlib.sha256(src[a:b].encode()).hexdigest()


def assembly_source_hash():
    """sha256 of the assembly sources (the tile kernel and the tile construction)."""
    import hashlib
    h = hashlib.sha256()
    for name in ("element.hip", "ctx.cpp"):
        with open(os.path.join(ROOT, "paper_0809_4802_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload, phase):
    """HBM-side bytes per launch of a phase's kernel from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, each scaled by the same counter on a copy of known size);
    None when there is none or the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{workload}_{phase}_traffic.json")
    if not os.path.exists(path):
        return None, None
    with open(path) as f:
        d = json.load(f)
    current = {"spmv": spmv_source_hash, "condense": assembly_source_hash}.get(phase)
    if current is None or d.get("source_sha256") != current():
        return None, os.path.relpath(path, ROOT) + " (stale: kernel changed since the counters were taken)"
    return d["traffic_bytes_per_launch"], os.path.relpath(path, ROOT)


def counter_run(B, cfg, mesh, u0, beta0, bc, dev):
    """One condensed assembly of the workload (mixed precision; transient workloads take their
    first backward-Euler step from the initial state), GMRES(50) + block-Jacobi on it capped at
    COUNTER_ITERS Arnoldi steps (as many launches of the Arnoldi SpMV), then one device-to-device
    copy of COPY_MIB MiB.  Meant to run under rocprofv3 --pmc."""
    import torch
    ctx = B.Context(torch.from_numpy(mesh.xyz).to(dev), torch.from_numpy(mesh.tets).to(dev),
                    torch.from_numpy(bc.dofs).to(dev), precision=B.VMS_MIXED)
    u = torch.from_numpy(u0).to(dev)
    dt = cfg.dt if cfg.dt > 0 else 0.0
    A, rhs, _ = B.vms_condense_assemble(ctx, u, torch.from_numpy(beta0).to(dev), cfg.re, dt, u if dt > 0 else None)
    x = ctx.new_vec()
    _, info = B.vms_gmres_solve(ctx, A, rhs, x, B.solve_opts(restart=50, rtol=1e-14, max_iters=COUNTER_ITERS),
                                allow_noconv=True)
    src = torch.empty(COPY_MIB << 20, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    src.fill_(1)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"counter_run": True, "arnoldi_steps": int(info.iters), "copy_bytes": COPY_MIB << 20}))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def oracle_assembly_rate(n_sample, threads):
    """Oracle condensed-assembly rate (tangents/s) on the first n_sample elements of cavity32, in a
    child process with OMP_NUM_THREADS = threads (the OpenMP runtime reads it at load)."""
    code = ("import sys, time, json; sys.path.insert(0, %r)\n"
            "from workloads import build_workload\n"
            "from oracle import vms as O\n"
            "from oracle.element import element_residual_tangent\n"
            "cfg, m, u, b, bc = build_workload('cavity32')\n"
            "t = m.tets[:%d]\n"
            "t0 = time.perf_counter()\n"
            "R, K = element_residual_tangent(m.xyz, t, u, b[:%d], 1.0 / cfg.re)\n"
            "Ks, Rs = O.condense(R, K)\n"
            "O.assemble_matrix(t, m.n_nodes, Ks, bc.dofs)\n"
            "O.assemble_vector(t, m.n_nodes, Rs)\n"
            "print(json.dumps(time.perf_counter() - t0))\n") % (ROOT, n_sample, n_sample)
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, check=True)
    dt = json.loads(out.stdout.strip().splitlines()[-1])
    return n_sample / dt, dt


def cpu_baseline(mesh, u0, beta0, bc, cfg, n_sample, forms):
    """The oracle (quadrature element, condensation, CSR assembly, GMRES with block-Jacobi and
    modified Gram-Schmidt, Newton) timed on the host cores.  value: the same metric as the
    bench line, n_elems / t(condensed assembly), on the first n_sample elements (all by default)
    with every OpenMP thread; then the same on a smaller sample with one thread, one GMRES(50)
    cycle on the assembled cavity 32^3 system, the Newton solve of cavity 4^3 (Re 1) to 1e-10
    measured, and the cavity 32^3 time to 1e-8 extrapolated from the measured per-phase costs and
    the GPU FP64 solve's Newton and GMRES iteration counts."""
    import numpy as np
    from oracle import vms as O
    from oracle.element import element_residual_tangent
    from workloads import build_workload

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    n_sample = mesh.n_elems if n_sample <= 0 else min(n_sample, mesh.n_elems)
    tets = mesh.tets[:n_sample]
    t0 = time.perf_counter()
    R, K = element_residual_tangent(mesh.xyz, tets, u0, beta0[:n_sample], 1.0 / cfg.re)
    Ks, Rs = O.condense(R, K)
    A = O.assemble_matrix(tets, mesh.n_nodes, Ks, bc.dofs)
    b = -O.assemble_vector(tets, mesh.n_nodes, Rs)
    t_asm = time.perf_counter() - t0
    out = {"value": n_sample / t_asm, "unit": "condensed tangents/s", "cores": threads, "kind": "oracle",
           "sample": f"{n_sample} of {mesh.n_elems} elements, one condensed assembly at the initial state: "
                     f"quadrature element + condensation + CSR assembly ({t_asm:.1f} s)",
           "cpu_model": cpu_model(), "nproc": os.cpu_count()}
    st_n = min(8000, mesh.n_elems)
    rate1, dt1 = oracle_assembly_rate(st_n, 1)
    out["single_thread"] = {"value": rate1, "unit": "condensed tangents/s", "cores": 1,
                            "sample": f"{st_n} elements ({dt1:.1f} s)"}
    extra = {}
    if n_sample == mesh.n_elems:
        b[bc.dofs] = 0.0
        Minv = O.block_jacobi_inverse(A, mesh.n_nodes)
        t0 = time.perf_counter()
        res = O.gmres(A, b, restart=50, max_iters=50, rtol=1e-14, Minv_blocks=Minv)
        t_cyc = time.perf_counter() - t0
        extra["gmres50_cycle_s"] = t_cyc
        extra["gmres50_cycle_iters"] = int(res.iters)
        f = forms.get("fp64_bj")
        if f:
            # per Newton step: one assembly (as timed) and one residual evaluation (about the
            # element part of it); per GMRES iteration: the cycle time / 50
            per_iter = t_cyc / max(1, res.iters)
            est = f["newton_steps"] * 2 * t_asm + f["gmres_iters"] * per_iter
            extra["time_to_1e-8_cavity32_s"] = {
                "value": est, "kind": "extrapolation",
                "from": f"{f['newton_steps']} Newton steps x 2 assemblies ({t_asm:.2f} s each) + "
                        f"{f['gmres_iters']} GMRES iterations x {per_iter * 1e3:.1f} ms (the GPU FP64 solve's counts)"}
    cfg1, m1, u1, b1, bc1 = build_workload("cavity4")
    prob = O.Problem(m1.xyz, m1.tets, bc1.dofs, nu=1.0 / cfg1.re)
    t0 = time.perf_counter()
    _, _, lg = O.newton_solve(prob, u1, b1, tol=cfg1.newton_tol, linear="gmres", rtol=cfg1.linear_rtol)
    extra["time_to_1e-10_cavity4_s"] = {"value": time.perf_counter() - t0, "kind": "measured",
                                        "newton_steps": len(lg.rnorms) - 1,
                                        "gmres_iters": int(sum(lg.lin_iters))}
    out["extra"] = extra
    return out


if __name__ == "__main__":
    main()
