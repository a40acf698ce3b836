#!/usr/bin/env python
"""Benchmark of the implicit modal DG hot path on one MI355X.

A step is one implicit BDF2 time step of the whole hot path: p-multigrid
setup (diagonal-block assembly, batched PLU), Newton iterations, each solved by
FGMRES preconditioned with one p-multigrid V-cycle (block-Jacobi smoothing,
matrix-free level-0 products, coarsest GMRES), residuals and exact Jacobian
products.  Workload (default): Taylor-Green vortex, Navier-Stokes with BR2,
Re = 1600, M = 0.1, Pr = 0.71, periodic [0, 2pi]^3, 16^3 hexahedra, p = 3
(1,310,720 DOF), dt = 0.05, FP64 pMG 3-2-1 with 2 + 2 BJ sweeps, coarsest
GMRES(BJ) 30, FGMRES(40) to rtol 1e-8.

value = DOF x time steps / second (GDOF/s) over the timed steps, inputs
resident on the device.  One JSON line is printed.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GDOF/s DG J·v; time-step solve s, mixed vs FP64 pMG-FGMRES @ rel 1e-8"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6

WORKLOADS = {
    "tgv_p3_16": dict(n=(16, 16, 16), lo=(0, 0, 0), hi=(2 * math.pi,) * 3, p=3, mach=0.1, mu=1.0 / 1600, Pr=0.71,
                      curved=0.0, ic="tgv", dt=0.05, levels=[3, 2, 1], restart=40, rtol=1e-8,
                      desc="Taylor-Green NS/BR2 Re=1600 M=0.1 on a periodic 16^3 hex box, p=3, one BDF2 step dt=0.05, "
                           "FP64 pMG 3-2-1 (2+2 BJ sweeps, coarsest GMRES(BJ) 30), FGMRES(40) rtol 1e-8"),
    "tgv_p4_16_curved": dict(n=(16, 16, 16), lo=(0, 0, 0), hi=(2 * math.pi,) * 3, p=4, mach=0.01, mu=1.0 / 1600,
                             Pr=0.71, curved=0.05, ic="tgv", dt=0.05, levels=[4, 2, 1], restart=40, rtol=1e-8,
                             # the FP64 unsteady residual bottoms out near 1e-7 of its initial value at
                             # M = 0.01 (fluxes of size p0 |u| ~ 1e5 ||R|| are rounded): Newton stops at
                             # 1e-6, the linear solves still go to 1e-8
                             newton_rtol=1e-6,
                             desc="Taylor-Green NS/BR2 M=0.01 on a curved 16^3 hex mesh, p=4, one BDF2 step, "
                                  "pMG 4-2-1, FGMRES(40) rtol 1e-8, Newton to 1e-6 of the initial residual"),
    "vortex_p2_4": dict(n=(4, 4, 4), lo=(0, 0, 0), hi=(10.0,) * 3, p=2, mach=0.5, mu=0.0, Pr=0.72, curved=0.0,
                        ic="vortex", dt=0.1, levels=[2], restart=30, rtol=1e-10,
                        desc="isentropic vortex Euler p=2 on a periodic 4^3 box, one BDF2 step dt=0.1, "
                             "FGMRES(30) + element block-Jacobi, rtol 1e-10"),
}


def make_case(wl_name):
    """Context and projected initial state of a workload."""
    import torch
    from paper_1812_04789_amd import binding, inputs
    wl = WORKLOADS[wl_name]
    vtx = inputs.box_vertices(wl["n"], wl["lo"], wl["hi"], amp=wl["curved"]) if wl["curved"] else None
    ctx = binding.Context(wl["n"], wl["lo"], wl["hi"], wl["p"], gamma=1.4, mu=wl["mu"], Pr=wl["Pr"], eta=7.0,
                          vertices=vtx)
    xq = ctx.quad_points().cpu().numpy()
    if wl["ic"] == "tgv":
        vals = inputs.taylor_green(xq, mach=wl["mach"])
    else:
        vals = inputs.isentropic_vortex(xq, mach=wl["mach"])
    W0 = ctx.project(torch.tensor(vals.reshape(-1), device="cuda"))
    if wl["ic"] == "vortex":
        W0 += torch.tensor(inputs.uniform_noise((ctx.ne, 5, ctx.nv), 1812, 1e-6).reshape(-1), device="cuda")
    return wl, ctx, W0


def popts_for(wl, mixed, coarse):
    from paper_1812_04789_amd import binding
    if mixed:
        return binding.pmg_opts(wl["levels"], prec_fine=binding.DG_FP32, prec_coarse=binding.DG_BF16,
                                coarse_matrix_free=coarse)
    return binding.pmg_opts(wl["levels"], prec_fine=binding.DG_FP64, prec_coarse=binding.DG_FP64,
                            coarse_matrix_free=coarse)


def time_steps(wl, ctx, W0, popts, nsteps, warmup):
    """`warmup` untimed then `nsteps` timed consecutive BDF2 steps from W0 (the
    first step of each run takes W^{n-1} = W^n); returns (seconds per step,
    final state, per-step statistics)."""
    import torch
    from paper_1812_04789_amd import binding
    fopts = binding.fgmres_opts(restart=wl["restart"], rtol=wl["rtol"])

    def run_steps(K):
        Wn, Wnm1 = W0.clone(), None
        stats = []
        for _ in range(K):
            Wnp1, st = ctx.bdf2_step(Wn, Wnm1, wl["dt"], popts, fopts, newton_rtol=wl.get("newton_rtol", 1e-10))
            stats.append(st)
            Wnm1, Wn = Wn, Wnp1
        return Wn, stats

    if warmup:
        run_steps(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    W, st = run_steps(nsteps)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / nsteps, W, st


def kernel_families(ctx, wl, W0, popts):
    """Per-family device time of one instrumented step (HIP events on the
    library stream, eager launches), with the library's algorithmic bytes and
    flops per launch."""
    ctx.timing(True)
    time_steps(wl, ctx, W0, popts, 1, 0)
    kern = ctx.timing_read()
    ctx.timing(False)
    fams = {}
    for kind, (ms, cnt, by, fl) in kern.items():
        if cnt == 0:
            continue
        fams[kind] = dict(ms_total=ms, launches=cnt, ms_avg=ms / cnt, bytes_per_launch=by / cnt,
                          gbs=(by / (ms * 1e-3) / 1e9) if (by and ms > 0) else None,
                          tflops=(fl / (ms * 1e-3) / 1e12) if (fl and ms > 0) else None)
    return fams


def step_summary(wl, ctx, W0, nsteps, warmup, coarse):
    """FP64 and mixed-precision steps of one workload: seconds per step, the
    speed-up, solver statistics and the distance between the two solutions."""
    t64, W64, st64 = time_steps(wl, ctx, W0, popts_for(wl, False, coarse), nsteps, warmup)
    out = {"fp64": t64, "newton": [s_.newton for s_ in st64], "fgmres_iters": [s_.linear_iters for s_ in st64],
           "max_rel_res_true": max(s_.max_rel_res_true for s_ in st64),
           "setup_s": float(sum(s_.setup_seconds for s_ in st64) / len(st64))}
    if len(wl["levels"]) > 1 or wl["p"] > 1:
        t32, W32, st32 = time_steps(wl, ctx, W0, popts_for(wl, True, coarse), nsteps, min(warmup, 1))
        out.update({"mixed": t32, "speedup": t64 / t32,
                    "mixed_newton": [s_.newton for s_ in st32],
                    "mixed_fgmres_iters": [s_.linear_iters for s_ in st32],
                    "mixed_max_rel_res_true": max(s_.max_rel_res_true for s_ in st32),
                    "mixed_vs_fp64_rel": (W32 - W64).norm().item() / W64.norm().item()})
    return out


def roofline_of(fams, dom, ctx, popts, workload):
    f = fams[dom]
    kname = kernel_name(dom, ctx.p, popts)
    if dom in ("lu", "diag_blocks"):
        return dict(kernel=kname, family=dom, bound="alu", achieved=f["tflops"], peak=FP64_PEAK_TFS,
                    unit="TFLOP/s", frac=(f["tflops"] or 0.0) / FP64_PEAK_TFS, traffic=None, ms_avg=f["ms_avg"])
    return dict(kernel=kname, family=dom, bound="hbm", achieved=f["gbs"], peak=HBM_PEAK_GBS, unit="GB/s",
                frac=f["gbs"] / HBM_PEAK_GBS, traffic=measured_traffic(kname, workload),
                ms_avg=f["ms_avg"], bytes_per_launch=f["bytes_per_launch"])


def jvp_rates(ctx, W0, reps):
    """FD product of Eq. DG-mf, exact product and residual: call time (HIP
    events around `reps` calls) and kernel time (the library's events)."""
    import torch
    from paper_1812_04789_amd import inputs
    v = torch.tensor(inputs.random_vector(ctx.ne, ctx.p, seed=7).reshape(-1), device="cuda")
    RW = ctx.residual(W0)
    y = ctx.empty()
    s = torch.cuda.current_stream()
    jv = {}
    for name, fn in (("fd", lambda: ctx.jvp(W0, RW, v, 30.0, y)), ("exact", lambda: ctx.jvp_exact(W0, v, 30.0, y)),
                     ("residual", lambda: ctx.residual(W0, y))):
        for _ in range(3):
            fn()
        ctx.timing(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            fn()
        e1.record(s)
        e1.synchronize()
        kk = ctx.timing_read()
        ctx.timing(False)
        kname = {"fd": "jvp_fd", "exact": "jvp_exact", "residual": "residual"}[name]
        kms, kc = kk[kname][0], kk[kname][1]
        jv[name] = dict(call_ms=e0.elapsed_time(e1) / reps, kernel_ms=kms / max(kc, 1),
                        gdof_s=ctx.ndof / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9)
        by = {"fd": 32.0, "exact": 24.0, "residual": 16.0}[name] * ctx.ndof
        jv[name]["kernel_gbs"] = by / (jv[name]["kernel_ms"] * 1e-3) / 1e9
        jv[name]["hbm_frac"] = jv[name]["kernel_gbs"] / HBM_PEAK_GBS
    # cold FD product: a 512 MB write between calls evicts the 256 MB last-level
    # cache, so W, v, R(W) and the neighbour reads come from HBM (kernel time only)
    flush = torch.empty(64 << 20, dtype=torch.float64, device="cuda")
    ctx.timing(True)
    for _ in range(10):
        flush.fill_(1.0)
        ctx.jvp(W0, RW, v, 30.0, y)
    torch.cuda.synchronize()
    kk = ctx.timing_read()
    ctx.timing(False)
    del flush
    kms = kk["jvp_fd"][0] / max(kk["jvp_fd"][1], 1)
    jv["fd_cold"] = dict(kernel_ms=kms, gdof_s=ctx.ndof / (kms * 1e-3) / 1e9,
                         kernel_gbs=32.0 * ctx.ndof / (kms * 1e-3) / 1e9,
                         hbm_frac=32.0 * ctx.ndof / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS)
    return jv


def jvp_only(args):
    """Only the products of the workload (for kernel profiles): `--jvp-reps`
    FD products, exact products and residuals, one JSON line of their rates."""
    import torch
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        calibrate_copy()
    wl, ctx, W0 = make_case(args.workload)
    jv = jvp_rates(ctx, W0, args.jvp_reps)
    print(json.dumps({"workload": args.workload, "ndof": ctx.ndof, "jvp": jv}), flush=True)
    ctx.close()


def paper_config_steps(args, nsteps):
    """ESDIRK3 steps of the 16^3 p = 3 Taylor-Green workload with the paper's
    preconditioner (FP64, and mixed: FP32 fine factors, BF16 coarse
    operators), seconds per step and iteration counts."""
    import torch
    from paper_1812_04789_amd import binding
    wl, ctx, W0 = make_case("tgv_p3_16")
    fopts = binding.fgmres_opts(restart=wl["restart"], rtol=wl["rtol"])
    out = {"scheme": "ESDIRK3, MG_full 3-2-1, GMRES(BJ) 10/10, coarsest GMRES(BILU-MDF) 30", "steps": nsteps}
    for tag, pf, pc in (("fp64", binding.DG_FP64, binding.DG_FP64), ("mixed", binding.DG_FP32, binding.DG_BF16)):
        popts = binding.paper_pmg_opts(wl["levels"], prec_fine=pf, prec_coarse=pc,
                                       coarsest_prec=binding.COARSEST_BILU)
        ctx.esdirk3_step(W0, wl["dt"], popts, fopts)              # warm-up (allocations)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        W, st = W0, None
        its, newt, worst = [], [], 0.0
        for _ in range(nsteps):
            W, st = ctx.esdirk3_step(W, wl["dt"], popts, fopts)
            its.append(st.linear_iters)
            newt.append(st.newton)
            worst = max(worst, st.max_rel_res_true)
        torch.cuda.synchronize()
        out[tag] = (time.perf_counter() - t0) / nsteps
        # per-family device time of one more (instrumented) step
        ctx.timing(True)
        ctx.esdirk3_step(W0, wl["dt"], popts, fopts)
        torch.cuda.synchronize()
        kern = ctx.timing_read()
        ctx.timing(False)
        out[tag + "_kernels_ms"] = {k: round(v[0], 3) for k, v in kern.items() if v[1]}
        out[tag + "_fgmres_iters"] = its
        out[tag + "_newton"] = newt
        out[tag + "_max_rel_res_true"] = worst
    out["speedup"] = out["fp64"] / out["mixed"]
    ctx.close()
    return out


_T0 = time.perf_counter()


def progress(stage):
    """One line on stderr as each stage of the run ends (the result lines stay
    on stdout)."""
    print("# bench: %s done at %.1f s" % (stage, time.perf_counter() - _T0), file=sys.stderr, flush=True)


def run(args):
    import torch

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        calibrate_copy()
    wl, ctx, W0 = make_case(args.workload)
    popts64 = popts_for(wl, False, args.coarse)

    # ---- timed FP64 steps of the workload: `value` ------------------------------------
    elapsed, W64, st64 = time_steps(wl, ctx, W0, popts64, args.steps, args.warmup)
    value = ctx.ndof / elapsed / 1e9
    steps_out = {args.workload: {"fp64": elapsed, "newton": [s_.newton for s_ in st64],
                                 "fgmres_iters": [s_.linear_iters for s_ in st64],
                                 "max_rel_res_true": max(s_.max_rel_res_true for s_ in st64),
                                 "setup_s": float(sum(s_.setup_seconds for s_ in st64) / len(st64))}}
    fams = kernel_families(ctx, wl, W0, popts64)
    dom = max(fams, key=lambda k: fams[k]["ms_total"]) if fams else None
    roof = roofline_of(fams, dom, ctx, popts64, args.workload) if dom else None
    progress("FP64 steps of " + args.workload)

    # ---- mixed-precision steps of the same workload ------------------------------------
    fams32 = None
    if not args.no_mixed:
        popts32 = popts_for(wl, True, args.coarse)
        t32, W32, st32 = time_steps(wl, ctx, W0, popts32, args.steps, min(args.warmup, 1))
        steps_out[args.workload].update({
            "mixed": t32, "speedup": elapsed / t32, "mixed_newton": [s_.newton for s_ in st32],
            "mixed_fgmres_iters": [s_.linear_iters for s_ in st32],
            "mixed_max_rel_res_true": max(s_.max_rel_res_true for s_ in st32),
            "mixed_vs_fp64_rel": (W32 - W64).norm().item() / W64.norm().item()})
        fams32 = kernel_families(ctx, wl, W0, popts32)
        progress("mixed steps of " + args.workload)

    # ---- J.v throughput -----------------------------------------------------------------
    jv = jvp_rates(ctx, W0, args.jvp_reps)
    ndof, ne, pdeg = ctx.ndof, ctx.ne, ctx.p
    progress("J.v rates")
    ctx.close()
    del W0, W64
    torch.cuda.empty_cache()
    if args.workload == "tgv_p3_16" and not args.no_large_jvp:
        jv["fd_32cube"] = large_jvp()
    if not args.no_matrix_based and args.workload == "tgv_p3_16":
        jv["matrix_based"] = matrix_based_jvp(WORKLOADS[args.workload])
    progress("large and matrix-based J.v")

    # ---- the paper's own solver configuration on the same workload ------------------------
    # ESDIRK3 (Sec. 4) with the preconditioner lagged over the step, full
    # multigrid (Alg. 1), GMRES(BJ) 10/10 smoothers and a 30-step coarsest
    # GMRES preconditioned by block ILU(0) in MDF order (Table MGSettings).
    if args.workload == "tgv_p3_16" and not args.no_paper_config:
        steps_out["tgv_p3_16_paper_config"] = paper_config_steps(args, max(1, min(args.steps, args.c3_steps)))
        progress("ESDIRK3 steps with the paper's preconditioner")

    # ---- the curved p = 4 low-Mach workload, FP64 and mixed -----------------------------
    if args.workload == "tgv_p3_16" and not args.no_c3:
        wl3, ctx3, W3 = make_case("tgv_p4_16_curved")
        k3 = max(1, min(args.steps, args.c3_steps))
        steps_out["tgv_p4_16_curved"] = step_summary(wl3, ctx3, W3, k3, 1, args.coarse)
        steps_out["tgv_p4_16_curved"]["steps"] = k3
        ctx3.close()
        del W3
        torch.cuda.empty_cache()
        progress("curved p = 4 steps")

    # ---- batching (96 independent cases) and serving (Poisson request stream) ----------
    batch = None
    if not args.no_batch and args.workload == "tgv_p3_16":
        batch = batch_bench(args)
        progress("batch")
    serving = None
    if not args.no_serving and args.workload == "tgv_p3_16" and args.serve_count > 0:
        from paper_1812_04789_amd import serve
        serving = serve.run(count=args.serve_count, rate=200.0, seed=1812, slots=args.serve_slots)
        # the same stream offered below saturation: latency without queueing
        serving["below_saturation"] = serve.run(count=40, rate=4.0, seed=1813, slots=args.serve_slots)
        serving["sustainable"] = sustainable_rate(args)
        progress("serving")

    # ---- CPU baseline: the oracle on a bounded sample ---------------------------------
    cpu = None
    if not args.no_cpu_baseline and args.workload == "tgv_p3_16":
        cpu = cpu_baseline()
        progress("CPU baseline")

    # Full detail first (one line), then the compact result line the driver reads.
    detail = {"kernels_fp64": fams, "kernels_mixed": fams32, "jvp": jv, "time_step": steps_out,
              "cpu_baseline": cpu, "batch": batch, "serving": serving,
              "kernel_timing_note": "kernel families timed with HIP events on the library stream over one "
                                    "instrumented step (eager launches); step times are from the "
                                    "un-instrumented steps"}
    print("# detail " + json.dumps(detail), flush=True)

    def r3(x):
        return None if x is None else float("%.4g" % x)

    ts = {}
    for k, d in steps_out.items():
        ts[k] = {kk: (r3(vv) if isinstance(vv, float) else vv) for kk, vv in d.items()
                 if kk in ("fp64", "mixed", "speedup", "newton", "fgmres_iters", "max_rel_res_true",
                           "mixed_max_rel_res_true", "mixed_vs_fp64_rel", "steps", "fp64_fgmres_iters")}
        for kk in ("newton", "fgmres_iters"):
            if kk in ts[k] and len(set(ts[k][kk])) <= 2:
                ts[k][kk] = sorted(set(ts[k][kk]))
    jsum = {"fd_gdof_s": r3(jv["fd"]["gdof_s"]), "fd_kernel_ms": r3(jv["fd"]["kernel_ms"]),
            "fd_hbm_frac": r3(jv["fd"]["hbm_frac"]), "fd_cold_hbm_frac": r3(jv["fd_cold"]["hbm_frac"]),
            "exact_gdof_s": r3(jv["exact"]["gdof_s"]), "residual_gdof_s": r3(jv["residual"]["gdof_s"])}
    if "fd_32cube" in jv:
        jsum["fd_32cube_hbm_frac"] = r3(jv["fd_32cube"]["hbm_frac"])
    # the FD product's FP64 work per launch is above the ridge (78.6 TFLOP/s / 8 TB/s):
    # its roofline is the FP64 ALU one, with the HBM fraction beside it
    jk = kernel_name("jvp_fd", wl["p"], popts64)
    jflop = measured_flops(jk, args.workload)
    jroof = dict(kernel=jk, bound="alu" if jflop else "hbm",
                 achieved=r3(jflop / (jv["fd"]["kernel_ms"] * 1e-3) / 1e12) if jflop else r3(jv["fd"]["kernel_gbs"]),
                 peak=FP64_PEAK_TFS if jflop else HBM_PEAK_GBS, unit="TFLOP/s" if jflop else "GB/s",
                 frac=r3(jflop / (jv["fd"]["kernel_ms"] * 1e-3) / 1e12 / FP64_PEAK_TFS) if jflop
                 else r3(jv["fd"]["hbm_frac"]),
                 flop_per_launch=jflop, hbm_achieved_gbs=r3(jv["fd"]["kernel_gbs"]), hbm_frac=r3(jv["fd"]["hbm_frac"]),
                 traffic=measured_traffic(jk, args.workload), bytes_per_launch=32.0 * ndof)
    out = {
        "metric": METRIC, "value": value, "unit": "GDOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "ndof": ndof, "elements": ne, "p": pdeg,
                   "value_is": "DOF x BDF2 steps per second, FP64 pMG-FGMRES steps",
                   "coarse_operators": {0: "assembled", 1: "matrix-free", 2: "assembled coarsest"}[args.coarse],
                   "mixed": "FP32 fine block factors, BF16 coarse operators (FP32 accumulation)"},
        "time_step_s": ts,
        "mixed_speedup": ts[args.workload].get("speedup"),
        "jvp": jsum,
        "roofline": roof,
        "jvp_roofline": jroof,
        "cpu_baseline": None if cpu is None else {k: cpu[k] for k in ("value", "unit", "cores", "kind", "sample")},
    }
    if batch is not None:
        out["batch"] = {"cases": batch["cases"], "total_dof": batch["total_dof"],
                        "bdf2_step_s": r3(batch["bdf2_step"]["seconds"]),
                        "bdf2_gdof_s": r3(batch["bdf2_step"]["gdof_s"]),
                        "fd_jvp_gdof_s": r3(batch["jvp"]["jvp_fd"]["gdof_s"])}
    if serving is not None:
        out["serving"] = {"rate_req_s": serving["rate_req_s"], "throughput_req_s": r3(serving["throughput_req_s"]),
                          "latency_p50_s": r3(serving["latency_s"]["p50"]),
                          "latency_p99_s": r3(serving["latency_s"]["p99"]),
                          "aggregate_gdof_s": r3(serving["aggregate_gdof_s"]),
                          "max_sustained_req_s": serving["sustainable"]["max_sustained_req_s"]}
    print(json.dumps(out), flush=True)


def large_jvp():
    """FD product on the 32^3 p=3 Taylor-Green mesh (10.5 M DOF, 335 MB per
    product: larger than the last-level cache), kernel time over 20 calls."""
    import torch
    from paper_1812_04789_amd import binding, inputs
    L = 2 * math.pi
    c = binding.Context((32, 32, 32), (0, 0, 0), (L, L, L), 3, gamma=1.4, mu=1.0 / 1600, Pr=0.71, eta=7.0)
    W = c.project(torch.tensor(inputs.taylor_green(c.quad_points().cpu().numpy(), mach=0.1).reshape(-1),
                               device="cuda"))
    v = torch.tensor(inputs.random_vector(c.ne, 3, seed=7).reshape(-1), device="cuda")
    RW = c.residual(W)
    y = c.empty()
    for _ in range(3):
        c.jvp(W, RW, v, 30.0, y)
    c.timing(True)
    for _ in range(20):
        c.jvp(W, RW, v, 30.0, y)
    torch.cuda.synchronize()
    kk = c.timing_read()
    c.timing(False)
    kms = kk["jvp_fd"][0] / max(kk["jvp_fd"][1], 1)
    out = dict(ndof=c.ndof, kernel_ms=kms, gdof_s=c.ndof / (kms * 1e-3) / 1e9,
               kernel_gbs=32.0 * c.ndof / (kms * 1e-3) / 1e9,
               hbm_frac=32.0 * c.ndof / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS)
    c.close()
    return out


def matrix_based_jvp(wl):
    """The matrix-based alternative to Eq. DG-mf on the benchmark mesh: K =
    shift M + dR/dW assembled once (diagonal + six face blocks per element,
    FP64) and applied by the 7-block product; call time over 5 products, in a
    context of its own so its ~47 GB are released afterwards."""
    import torch
    from paper_1812_04789_amd import binding, inputs
    c = binding.Context(wl["n"], wl["lo"], wl["hi"], wl["p"], gamma=1.4, mu=wl["mu"], Pr=wl["Pr"], eta=7.0)
    W = c.project(torch.tensor(inputs.taylor_green(c.quad_points().cpu().numpy(), mach=wl["mach"]).reshape(-1),
                               device="cuda"))
    v = torch.tensor(inputs.random_vector(c.ne, c.p, seed=7).reshape(-1), device="cuda")
    t0 = time.perf_counter()
    c.assemble_operator(W, 30.0)
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t0
    y = c.empty()
    c.jvp_assembled(v, y)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(5):
        c.jvp_assembled(v, y)
    e1.record(s)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / 5
    nb = 5 * c.nv
    by = c.ne * (7.0 * nb * nb * 8 + 16.0 * nb)
    out = dict(assemble_s=t_asm, call_ms=ms, gdof_s=c.ndof / (ms * 1e-3) / 1e9, gbs=by / (ms * 1e-3) / 1e9,
               hbm_frac=by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, operator_gb=by / 1e9)
    c.close()
    return out


def batch_bench(args):
    """The 96-case batch: one persistent launch of the FD / exact product over
    every case (default and autotuned tiles) against one launch per case, and
    one mixed-precision BDF2 step of every case."""
    import numpy as np
    import torch
    from paper_1812_04789_amd import binding, inputs, serve
    wl = inputs.batch_cases()
    gas = serve.GAS
    b = binding.Batch([dict(c, **gas) for c in wl])
    W0 = []
    for i, c in enumerate(wl):
        ctx = b.case(i)
        ks, ph = inputs.fourier_phases(c["seed"])
        W0.append(ctx.project(inputs.fourier_state_torch(ctx.quad_points(), ks, ph, gamma=gas["gamma"],
                                                         mach=c["mach"]).reshape(-1)))
    W0 = torch.cat(W0)
    v = torch.tensor(np.random.default_rng(7).standard_normal(b.ndof), device="cuda")
    R = b.residual(W0)
    y = b.empty()
    s = torch.cuda.current_stream()

    def timed(fn, reps):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            fn()
        e1.record(s)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {"cases": len(wl), "total_dof": b.ndof, "elements": int(sum(np.prod(c["n"]) for c in wl)),
           "degrees": {str(p): sum(1 for c in wl if c["p"] == p) for p in (1, 2, 3, 4)}}
    reps = args.jvp_reps
    jv = {}
    for kind, fn in (("jvp_fd", lambda: b.jvp(W0, R, v, 30.0, y)), ("jvp_exact", lambda: b.jvp_exact(W0, v, 30.0, y))):
        ms_default = timed(fn, reps)
        tile_default = b.tile(kind)
        tuned = b.tune(kind, W0, R, v, reps=3)
        ms_tuned = timed(fn, reps)
        jv[kind] = {"ms_default_tile": ms_default, "default_tile": tile_default, "ms_tuned": ms_tuned,
                    "tuned_tile": tuned, "gdof_s": b.ndof / (ms_tuned * 1e-3) / 1e9}
    # the same products as one launch per case (plain contexts on the same stream)
    singles = [binding.Context(c["n"], c["lo"], c["hi"], c["p"], **gas) for c in wl]
    Ws, Rs, vs, ys = b.split(W0), b.split(R), b.split(v), b.split(y)
    ms_sep = timed(lambda: [ctx.jvp(Ws[i], Rs[i], vs[i], 30.0, ys[i]) for i, ctx in enumerate(singles)], 5)
    for ctx in singles:
        ctx.close()
    jv["jvp_fd"]["ms_one_launch_per_case"] = ms_sep
    jv["jvp_fd"]["batching_speedup"] = ms_sep / jv["jvp_fd"]["ms_tuned"]
    out["jvp"] = jv
    # one BDF2 step of every case, mixed precision, cases concurrent on worker streams
    popts = [serve.solver_opts(c["p"], True)[0] for c in wl]
    fopts = binding.fgmres_opts(restart=40, rtol=1e-8)
    nw = args.batch_workers
    b.bdf2_step(W0, None, 0.05, popts, fopts, workers=nw, raise_on_noconv=False)   # warm-up (allocations)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    W1, st, status = b.bdf2_step(W0, None, 0.05, popts, fopts, workers=nw, raise_on_noconv=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out["bdf2_step"] = {"seconds": el, "gdof_s": b.ndof / el / 1e9, "workers": nw, "status": status,
                        "max_rel_res_true": max(x.max_rel_res_true for x in st),
                        "newton_max": max(x.newton for x in st),
                        "linear_iters_mean": float(np.mean([x.linear_iters for x in st])),
                        "precision": "FP32 fine factors, BF16 assembled coarsest level"}
    b.close()
    return out


def kernel_name(family, p, popts):
    """HIP kernel behind a timing family in the FP64 run (for the profile cross-reference)."""
    if family == "bj_fine":
        return "lu_solve_blocked_kernel<double>" if 5 * (p + 1) ** 3 > 135 else "inv_gemv_kernel<double>"
    return {"residual": "dg_kernel<P,NS,CURVED,0>", "jvp_fd": "dg_kernel<P,NS,CURVED,1>",
            "jvp_exact": "dg_kernel<P,NS,CURVED,2>", "diag_blocks": "diag_kernel", "lu": "lu_blocked_kernel<double>",
            "bsr": "bsr_rows_kernel<double,double,UNIT,DOTS>", "bj_coarse": "inv_gemv_kernel<double>",
            "arnoldi": "gs_update_kernel + gs_update_normalise_kernel (+ gs_dots_kernel)"}.get(family, family)


def measured_traffic(kname, workload):
    """HBM bytes per launch of `kname` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary (profiles/traffic.txt), scaled by the copy-kernel
    calibration recorded there.  None when no entry matches this kernel and
    workload, or when the kernel's source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("#") or "=" not in line:
            continue
        kv = dict(t.split("=", 1) for t in line.split())
        if kv.get("kernel") != kname or kv.get("workload") != workload:
            continue
        src = os.path.join(ROOT, "paper_1812_04789_amd", "csrc", kv["source"])
        if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != kv["sha"]:
            return None
        return float(kv["bytes_per_launch"])
    return None


def measured_flops(kname, workload):
    """FP64 FLOP per launch of `kname` from the committed rocprofv3 instruction
    counts (profiles/flops_dg_tgv_p3_16.txt); None when no entry matches this
    kernel and workload, or when the kernel's source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "flops_dg_tgv_p3_16.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("#") or "=" not in line:
            continue
        kv = dict(t.split("=", 1) for t in line.split())
        if kv.get("kernel") != kname or kv.get("workload") != workload:
            continue
        src = os.path.join(ROOT, "paper_1812_04789_amd", "csrc", kv["source"])
        if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != kv["sha"]:
            return None
        return float(kv["flop_per_launch"])
    return None


def calibrate_copy():
    """A plain device copy of 1 GiB (read 1 GiB, write 1 GiB): the reference
    dispatch for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE counts to bytes."""
    import torch
    x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    del x, y


def sustainable_rate(args, rates=(6.0, 10.0, 12.0, 14.0, 18.0, 22.0, 26.0, 30.0), seconds=8.0):
    """The same kind of request stream offered at increasing rates below the
    200 req/s of the workload, each for `seconds` of arrivals (at least 60
    requests): a rate is sustained when the queue does not grow over the run
    (the median queueing time of the last third of the requests stays within
    twice that of the first third, or below the median service time).
    Returns each probe's figures and the highest sustained rate."""
    from paper_1812_04789_amd import serve
    probes = []
    best = None
    for r in rates:
        count = max(60, int(round(r * seconds)))
        out = serve.run(count=count, rate=r, seed=1814, slots=args.serve_slots)
        q0, q1 = out["queue_s"]["first_third_p50"], out["queue_s"]["last_third_p50"]
        ok = q1 <= max(2.0 * q0, out["service_s"]["p50"])
        probes.append({"rate_req_s": r, "requests": count, "throughput_req_s": out["throughput_req_s"],
                       "latency_p50_s": out["latency_s"]["p50"], "latency_p99_s": out["latency_s"]["p99"],
                       "queue_first_third_p50_s": q0, "queue_last_third_p50_s": q1,
                       "service_p50_s": out["service_s"]["p50"], "service_p99_s": out["service_s"]["p99"],
                       "aggregate_gdof_s": out["aggregate_gdof_s"], "sustained": ok})
        progress("serving probe at %.0f req/s" % r)
        if ok:
            best = r
        else:
            break
    return {"seconds_of_arrivals": seconds, "probes": probes, "max_sustained_req_s": best}


def cpu_baseline():
    """The oracle (plain NumPy FP64, as it stands) timed on the host: the
    residual and the FD product of Eq. DG-mf on (a) the whole 4^3 p = 2 Euler
    vortex mesh (8,640 DOF) and (b) a periodic 2 x 16 x 16 slab of the 16^3
    p = 3 Taylor-Green mesh (same element size and physics, the Taylor-Green
    field restricted to the slab; 163,840 DOF: the oracle is vectorised over elements, so its per-DOF rate on the
    slab is that of the whole mesh), each with NumPy/BLAS limited to one
    thread and with all of the host's threads.  `value` is the FD-product
    rate on the slab with all threads (GDOF/s, to set beside the GPU's J.v
    rate); `cores` is the CPU time over the wall time of that measurement,
    i.e. the threads the oracle actually kept busy."""
    import math as m
    import platform
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import mesh as omesh, dg as odg, linear as olin
    from paper_1812_04789_amd import inputs
    L = 2 * m.pi
    nproc = os.cpu_count()
    model = platform.processor() or ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    cases = {
        "vortex_p2_4": dict(mesh=omesh.BoxMesh((4, 4, 4), (0, 0, 0), (10, 10, 10)), p=2, mu=0.0, Pr=0.72,
                            ic=lambda x: inputs.isentropic_vortex(x, mach=0.5), reps=5),
        "tgv_p3_16_slab_2x16x16": dict(mesh=omesh.BoxMesh((2, 16, 16), (0, 0, 0), (L / 8, L, L)), p=3,
                                       mu=1.0 / 1600, Pr=0.71, ic=lambda x: inputs.taylor_green(x, mach=0.1), reps=3),
    }
    res = {}
    for name, c in cases.items():
        D = odg.Discretization(c["mesh"], c["p"], gamma=1.4, mu=c["mu"], Pr=c["Pr"], eta=7.0)
        W = D.project(c["ic"](D.quad_points()))
        v = inputs.random_vector(D.mesh.ne, c["p"], seed=7)
        RW = D.residual(W)
        for threads, tag in ((1, "1thread"), (nproc, "all")):
            with threadpool_limits(threads):
                for op, fn in (("residual", lambda: D.residual(W)), ("jvp_fd", lambda: olin.jvp_fd(D, W, RW, v, 30.0))):
                    walls, cpus = [], []
                    for _ in range(c["reps"]):
                        c0, t0 = time.process_time(), time.perf_counter()
                        fn()
                        walls.append(time.perf_counter() - t0)
                        cpus.append(time.process_time() - c0)
                    k = int(np.argsort(walls)[len(walls) // 2])
                    res["%s/%s/%s" % (name, op, tag)] = dict(seconds=walls[k], gdof_s=D.ndof() / walls[k] / 1e9,
                                                             busy_threads=cpus[k] / walls[k], ndof=D.ndof())
    main = res["tgv_p3_16_slab_2x16x16/jvp_fd/all"]
    return {"value": main["gdof_s"], "unit": "GDOF/s", "cores": max(1, int(round(main["busy_threads"]))),
            "kind": "oracle",
            "sample": "oracle FD J.v (Eq. DG-mf) on a periodic 2x16x16 slab of the 16^3 p=3 Taylor-Green NS mesh "
                      "(163,840 DOF), all %d host threads allowed (%.1f s); host: %s, nproc %d; also timed: "
                      "residual and FD J.v on one thread and on the whole 4^3 p=2 vortex mesh (detail line)"
                      % (nproc, main["seconds"], model, nproc),
            "host": {"model": model, "nproc": nproc}, "runs": res}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="tgv_p3_16", choices=sorted(WORKLOADS))
    ap.add_argument("--jvp-reps", type=int, default=30)
    ap.add_argument("--no-large-jvp", action="store_true", help="skip the 32^3 p=3 FD product")
    ap.add_argument("--no-matrix-based", action="store_true", help="skip the assembled-operator product")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the curved 16^3 p=4 M=0.01 workload's steps")
    ap.add_argument("--no-paper-config", action="store_true",
                    help="skip the ESDIRK3 steps with the paper's preconditioner (FMG, GMRES(BJ), BILU coarsest)")
    ap.add_argument("--c3-steps", type=int, default=3, help="timed steps of the curved p=4 workload (at most --steps)")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--batch-workers", type=int, default=16, help="host threads (and streams) of the batch step")
    ap.add_argument("--serve-count", type=int, default=400)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--jvp-only", action="store_true",
                    help="time only the FD / exact products and the residual of the workload (for profiles)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 1 GiB device copy first (reference dispatch for HBM counters)")
    ap.add_argument("--coarse", type=int, default=2, choices=[0, 1, 2],
                    help="coarse operators: 0 assembled, 1 matrix-free, 2 assembled on the coarsest level")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the hot path of this build is single-GPU "
              "(multi-GPU sharding is a design note, not implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.jvp_only:
        jvp_only(args)
    else:
        run(args)


if __name__ == "__main__":
    main()
