#!/usr/bin/env python3
"""Benchmark of the Parareal-over-stencils hot path on one MI355X.

One step = one pass of the whole hot path over the synthetic workload:
  * the serial fine reference u_fine = F_{P-1}(...F_0(u0)) (batched sweep kernel, batch 1)
  * the Parareal solve: start-up coarse run, K iterations of {batched F over all
    slices, coarse chain + FP64 correction + inter-iterate norms}, and the
    defect d^k against u_fine every iteration.
Inputs are resident in HBM before the timed region.  The JSON line reports the
fine-sweep GLUP/s of the whole step (fine lattice updates / wall time), the
roofline of the fused RK4 kernel measured with HIP events on the solve's
stream, the oracle's CPU rate on a bounded sample, and time-to-solution of the
batched solve against plain per-slice FP64 Parareal and serial FP64 fine.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c2_128_fp64]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# The paper's measured Parareal speedups (Table 1: K = 3, N_f/N_c = 16, one
# time slice per node on Piz Daint; CPU runs on 8-core Xeon E5-2670 nodes,
# GPU runs on one NVIDIA K20X per node).  Context only: another machine.
PAPER_TABLE1 = {"nodes": [4, 8, 16, 32, 64, 128],
                "S_measured_cpu": [1.3, 2.6, 5.0, 9.5, 17.6, 29.7],
                "S_measured_gpu": [1.3, 2.6, 5.0, 9.3, 16.6, 26.3]}

# HBM bytes per batched fused-RK4 launch measured with rocprofv3 FETCH_SIZE /
# WRITE_SIZE (scaled by the plain-copy calibration), for the kernel variant
# and workload they were taken on (the hbm_counters summaries).  Reported
# only while the plan still launches that variant.
MEASURED_TRAFFIC = {("rk4w_f64_x128_y8_p2x1_w16", "c2_128_fp64"): 558109929}


def kernel_of(variant):
    """HIP kernel that a fused fine variant launches."""
    for prefix, kernel in (("rk4w_", "rk4_step_rows"), ("rk4b_", "rk4_step_fused1b"), ("rk4c_", "rk4_step_fused1c"),
                           ("rk4_", "rk4_step_fused")):
        if variant.startswith(prefix):
            return kernel
    return "rk4_stage_ref"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(p, u0_np, budget_s=15.0):
    """Time the FP64 oracle's RK4 steps on the same grid (bounded sample)."""
    import oracle
    oracle.lib()
    t = time.perf_counter()
    oracle.fine_steps(p, 0, 1, u0_np)
    one = time.perf_counter() - t
    m = int(max(2, min(400, budget_s / max(one, 1e-6))))
    t = time.perf_counter()
    oracle.fine_steps(p, 0, m, u0_np)
    dt = time.perf_counter() - t
    return {"value": m * p.npts / dt / 1e9, "unit": "GLUP/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": "%d FP64 RK4 steps of the oracle on one %dx%dx%d field (%.1f s)" % (m, p.n[0], p.n[1], p.n[2],
                                                                                        dt)}


def copy_ceiling(pr, torch, nbytes):
    """Achievable HBM bandwidth of a plain copy of `nbytes` with the library's
    own streaming kernel (pr_copy_probe): best over its variants and grid
    sizes, each the best of three windows of 10 copies timed with HIP events
    on the current stream.  GB/s counts read + write bytes."""
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").normal_()
    b = torch.empty_like(a)
    best = (0.0, None)
    for variant in (0, 1, 2, 3):
        for bpc in (2, 4, 8, 16):
            pr.copy_probe(a, b, variant, bpc)
            torch.cuda.synchronize()
            t = float("inf")
            for _ in range(3):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(10):
                    pr.copy_probe(a, b, variant, bpc)
                e1.record()
                torch.cuda.synchronize()
                t = min(t, e0.elapsed_time(e1) / 10)
            gbs = 2 * nbytes / (t * 1e-3) / 1e9
            if gbs > best[0]:
                best = (gbs, (variant, bpc, t))
    ok = bool(torch.equal(a, b))
    del a, b
    torch.cuda.empty_cache()
    gbs, (variant, bpc, t) = best
    return {"gbs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4), "bytes_copied": nbytes,
            "kernel": "copy_probe_kernel variant %d, %d blocks of 256 per CU" % (variant, bpc),
            "copy_us": round(t * 1e3, 2), "copy_exact": ok}


def per_config_rates(pr, W, torch, kernel_of):
    """Rate of the batched fine-step launch (all P slices in one launch) on
    every workload, timed with HIP events over a few steps on random data
    (outside the timed region); the batched workload runs a one-iteration
    timed plan over its 64 instances."""
    out = {}

    def ev_time(fn, steps):
        """best of three timed windows of `steps` launches, after one warm window"""
        fn(steps)
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn(steps)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1) / steps)
        return best

    for name in ("c1_32_fp64", "c2_128_fp64", "c3_256_mixed", "c5_512_mixed"):
        p, _ = W.config(name)
        mixed = W.MIXED[name]
        tdt = torch.float32 if mixed else torch.float64
        es = 4 if mixed else 8
        u = torch.randn((p.P,) + tuple(reversed(p.n)), dtype=tdt, device="cuda")
        o = torch.empty_like(u)
        steps = 128 if p.npts * p.P < (1 << 27) else (16 if p.npts * p.P < (1 << 30) else 4)
        ms = ev_time(lambda k: pr.fine_sweep(p, u, [s * p.nf for s in range(p.P)], k, u_out=o), steps)
        lups = p.P * p.npts
        fv = pr.sweep_kernel_variant(p, pr.PR_FP32 if mixed else pr.PR_FP64, p.P, 0)
        out[name] = {"glups": round(lups / ms / 1e6, 1), "gbs": round(lups * 2 * es / ms / 1e6, 1),
                     "frac": round(lups * 2 * es / ms / 1e6 / HBM_PEAK_GBS, 4),
                     "launch_us": round(ms * 1e3, 1), "kernel": "%s (%s)" % (kernel_of(fv), fv)}
        del u, o
        torch.cuda.empty_cache()
    # the paper's own setup (Section 3.1): fourth-order F on 128^3 FP64, all
    # 8 slices per launch
    pp = W.paper_setup(100.0)
    u = torch.randn((pp.P,) + tuple(reversed(pp.n)), dtype=torch.float64, device="cuda")
    o = torch.empty_like(u)
    ms = ev_time(lambda k: pr.fine_sweep(pp, u, [s * pp.nf for s in range(pp.P)], k, u_out=o), 32)
    lups = pp.P * pp.npts
    fv = pr.sweep_kernel_variant(pp, pr.PR_FP64, pp.P, 0)
    out["paper_setup_order4_fp64"] = {"glups": round(lups / ms / 1e6, 1), "gbs": round(lups * 16 / ms / 1e6, 1),
                                      "frac": round(lups * 16 / ms / 1e6 / HBM_PEAK_GBS, 4),
                                      "launch_us": round(ms * 1e3, 1), "kernel": "%s (%s)" % (kernel_of(fv), fv)}
    del u, o
    torch.cuda.empty_cache()
    insts = W.batched_config(64)
    probs = [W.Problem(**{**q.__dict__, "K": 1}) for q, _ in insts]
    u0s = [torch.randn(tuple(reversed(q.n)), dtype=torch.float64, device="cuda") for q in probs]
    plan = pr.Plan(probs, pr.PR_MODE_MIXED | pr.PR_MODE_TIMED)
    plan.solve(u0s, want_log=False)
    plan.solve(u0s, want_log=False)
    tm = plan.timings()
    # F launches of the plan: step j covers the slices with more than j steps
    lups = sum(q.P * q.npts * q.nf for q in probs)
    out["c4_batched_64"] = {"glups": round(lups / tm["fine_ms"] / 1e6, 1),
                            "gbs": round(lups * 8 / tm["fine_ms"] / 1e6, 1),
                            "frac": round(lups * 8 / tm["fine_ms"] / 1e6 / HBM_PEAK_GBS, 4),
                            "fine_launches": int(tm["fine_launches"]),
                            "kernel": "%s (%s)" % (kernel_of(plan.kernel_variants()[0]), plan.kernel_variants()[0]),
                            "launch_groups": [{"variant": v, "instances": n} for v, _, n in plan.fine_groups()]}
    del plan, u0s
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2_128_fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--mixed-config", default="c3_256_mixed",
                    help="workload of the batched-FP32 vs plain-per-slice-FP64 comparison ('' to skip)")
    ap.add_argument("--no-per-config", action="store_true",
                    help="skip the per-workload F kernel rates (all five workloads)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain device-to-device copy of this size first (calibrates HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (the time slices would shard "
              "across GPUs, with the coarse-chain hand-off sent over xGMI). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1409_8563_amd as pr
    import workloads as W
    from paper_1409_8563_amd import costmodel

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    pr.lib()
    p, modes = W.config(args.config)
    mixed = W.MIXED[args.config]
    sdt = torch.float32 if mixed else torch.float64
    es = 4 if mixed else 8
    mode = pr.PR_MODE_MIXED if mixed else pr.PR_MODE_FP64
    log("config", args.config, "n", p.n, "P", p.P, "K", p.K, "nt_fine", p.nt_fine, "nt_coarse", p.nt_coarse)

    if args.copy_probe_mib > 0:
        nbytes = args.copy_probe_mib << 20
        a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("copy probe: %d MiB device-to-device" % args.copy_probe_mib)
        del a, b

    u0_np = W.synth_u0(p.n, modes)
    u0 = torch.from_numpy(u0_np).cuda()
    u0s = u0.to(sdt)
    ufine = torch.empty_like(u0s)
    ufine64 = torch.empty_like(u0)
    uT = torch.empty_like(u0)
    plan = pr.Plan([p], mode | pr.PR_MODE_TIMED)
    torch.cuda.synchronize()

    def step():
        pr.fine_sweep(p, u0s, 0, p.nt_fine, u_out=ufine)          # serial fine reference
        ref = ufine if not mixed else ufine64.copy_(ufine)
        _, lg = plan.solve([u0], uT=[uT], ref=[ref])
        return lg

    for i in range(args.warmup):
        step()
        log("warmup", i + 1, "done")
    torch.cuda.synchronize()
    fine_ms = launches = 0.0
    t0 = time.perf_counter()
    for i in range(args.steps):
        lg = step()
        tm = plan.timings()
        fine_ms += tm["fine_ms"]
        launches += tm["fine_launches"]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    log("timed %d steps: %.2f ms/step" % (args.steps, ms_per_step))

    n3 = p.npts
    skip = bool(p.flags & W.SKIP_CONVERGED)
    fine_slices = sum((p.P - k) if skip else p.P for k in range(p.K))
    fine_lups = fine_slices * p.nf * n3 + p.nt_fine * n3
    value = fine_lups / (ms_per_step / 1e3) / 1e9

    # dominant kernel: the fused RK4 step over all slices of one iteration
    avg_launch_s = fine_ms / 1e3 / max(launches, 1)
    lups_per_launch = fine_slices * p.nf * n3 / max(launches / args.steps, 1)
    bytes_per_launch = 2 * es * lups_per_launch
    achieved = bytes_per_launch / avg_launch_s / 1e9
    dk = [float(lg[0, k, 8] / lg[0, k, 9]) for k in range(p.K)]
    fine_variant, coarse_variant = plan.kernel_variants()
    traffic = MEASURED_TRAFFIC.get((fine_variant, args.config))
    ceiling = copy_ceiling(pr, torch, int(bytes_per_launch) // 2)
    log("copy ceiling", ceiling)

    extra = {}
    if not args.no_per_config:
        extra["per_config_fine_kernel"] = per_config_rates(pr, W, torch, kernel_of)
        log("per-config F rates", extra["per_config_fine_kernel"])
    if not args.no_compare:
        # time-to-solution comparisons (outside the timed region)
        def timed(fn, reps=10, warm=3):
            """median wall time (ms) of reps calls after warm calls"""
            for _ in range(warm):
                fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                t = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                ts.append((time.perf_counter() - t) * 1e3)
            return float(np.median(ts))

        u64 = u0
        out64 = torch.empty_like(u64)
        t_batched = timed(lambda: plan.solve([u0], uT=[uT], want_log=False))
        plan_g = pr.Plan([p], mode | pr.PR_MODE_GRAPH)
        t0g = time.perf_counter()
        plan_g.solve([u0], uT=[uT], want_log=False)
        torch.cuda.synchronize()
        t_capture = (time.perf_counter() - t0g) * 1e3
        t_graph = timed(lambda: plan_g.solve([u0], uT=[uT], want_log=False))
        del plan_g
        plan_ps = pr.Plan([p], pr.PR_MODE_FP64 | pr.PR_MODE_PER_SLICE)
        t_plain = timed(lambda: plan_ps.solve([u0], uT=[uT], want_log=False))
        del plan_ps
        q = W.Problem(**dict(p.__dict__))
        q.flags |= W.SKIP_CONVERGED
        plan_sk = pr.Plan([q], mode)
        t_skip = timed(lambda: plan_sk.solve([u0], uT=[uT], want_log=False))
        del plan_sk
        t_serial = timed(lambda: pr.fine_sweep(p, u64, 0, p.nt_fine, u_out=out64), reps=5, warm=1)
        t_coarse = timed(lambda: pr.coarse_sweep(p, u64, 0, p.nt_coarse, u_out=out64), reps=5, warm=1)
        tau = (t_coarse / p.nt_coarse) / (t_serial / p.nt_fine)
        # the same ratio for the paper's own setup (fourth-order F, 128^3)
        pp = W.paper_setup(100.0)
        upp = torch.from_numpy(W.synth_u0(pp.n, W.single_mode((1, 1, 1)))).cuda()
        opp = torch.empty_like(upp)
        t_fp = timed(lambda: pr.fine_sweep(pp, upp, 0, 256, u_out=opp), reps=5, warm=1) / 256
        t_cp = timed(lambda: pr.coarse_sweep(pp, upp, 0, 64, u_out=opp), reps=5, warm=1) / 64
        tau_paper = t_cp / t_fp
        del upp, opp
        extra.update({
            "time_to_solution_ms": {"parareal_batched": round(t_batched, 3),
                                    "parareal_batched_graph_replay": round(t_graph, 3),
                                    "first_call_with_graph_capture": round(t_capture, 3),
                                    "parareal_batched_skip_converged": round(t_skip, 3),
                                    "parareal_plain_fp64_per_slice": round(t_plain, 3),
                                    "serial_fine_fp64": round(t_serial, 3)},
            "batched_vs_plain_fp64_speedup": round(t_plain / t_batched, 3),
            "tau_c_over_tau_f_fp64_serial": round(tau, 4),
            "S_bound_eq_speedup": round(costmodel.speedup_bound(p.P, p.K, p.nc / p.nf, tau), 3),
            # eq. speedup at the paper's K = 3 and N_f/N_c = 16 with this GPU's
            # measured coarse/fine step-cost ratio, beside the paper's Table 1
            "paper_table1_context": {
                "hardware": "Piz Daint (Cray XC30): CPU = 8-core Xeon E5-2670 per node, GPU = one NVIDIA K20X "
                            "per node; one time slice per node, K = 3, N_f/N_c = 16, 128^3",
                **PAPER_TABLE1,
                "tau_c_over_tau_f_paper_setup_this_gpu": round(tau_paper, 4),
                "S_bound_with_this_gpu_tau": [round(costmodel.speedup_bound(n, 3, 1.0 / 16.0, tau_paper), 2)
                                              for n in PAPER_TABLE1["nodes"]]},
        })
        # G on the grid coarsened by 2 (restriction, Euler steps with h = 2/n,
        # linear or cubic interpolation), with the smallest power-of-two coarse
        # count that the coarsened grid keeps stable
        ref64 = ufine if not mixed else ufine64.copy_(ufine)
        plan_k0 = pr.Plan([W.Problem(**{**p.__dict__, "K": 0})], mode)
        g_slice_plain = timed(lambda: plan_k0.solve([u0], uT=[uT], want_log=False), reps=5, warm=1) / p.P
        del plan_k0
        f_slice = t_serial / p.P
        coarsened = {}
        for label, extra_flags in (("linear", W.COARSEN_G), ("cubic", W.COARSEN_G | W.CUBIC_INTERP)):
            q = W.Problem(**dict(p.__dict__))
            q.flags = (q.flags | extra_flags) & ~W.SKIP_CONVERGED
            half = [v // 2 for v in q.n]
            q.nt_coarse = W.stable_coarse_steps(half, q.a, q.nu0, q.nu_amp, q.T, q.P, power_of_two=True,
                                                minimum=q.P)
            plan_c = pr.Plan([q], mode)
            t_c = timed(lambda: plan_c.solve([u0], uT=[uT], want_log=False), reps=5, warm=1)
            _, lg_c = plan_c.solve([u0], uT=[uT], ref=[ref64])
            del plan_c
            qk0 = W.Problem(**{**q.__dict__, "K": 0})
            plan_c0 = pr.Plan([qk0], mode)
            g_slice = timed(lambda: plan_c0.solve([u0], uT=[uT], want_log=False), reps=5, warm=1) / q.P
            del plan_c0
            r = g_slice / f_slice
            coarsened[label] = {
                "nt_coarse": q.nt_coarse, "time_to_solution_ms": round(t_c, 3),
                "G_over_F_per_slice": round(r, 4),
                "S_bound_eq_speedup": round(1.0 / ((1 + q.K / q.P) * r + q.K / q.P), 3),
                "defect_dk": [float("%.3e" % (lg_c[0, k, 8] / lg_c[0, k, 9])) for k in range(q.K)]}
        extra["coarsened_G"] = {"plain_G_over_F_per_slice": round(g_slice_plain / f_slice, 4), **coarsened}
        log("comparisons", extra)
        if args.mixed_config:
            # batched FP32-sweep Parareal against plain per-slice FP64 Parareal on
            # the same workload.  Errors are taken on the device against the FP64
            # serial fine solution of the library's own FP64 path (that path is
            # checked against the CPU oracle by the parity tests), and between the
            # two Parareal results (the FP32 sweeps' own rounding).
            pm, mm = W.config(args.mixed_config)
            um = torch.from_numpy(W.synth_u0(pm.n, mm)).cuda()
            u_fine64 = pr.fine_sweep(pm, um, 0, pm.nt_fine)
            uT_mixed = torch.empty_like(um)
            uT_plain = torch.empty_like(um)

            def errs(x, r):
                o = pr.defect_norm(x, r).cpu().numpy()[0]
                return {"max_abs": float("%.3e" % o[0]), "rel_l2": float("%.3e" % np.sqrt(o[2] / o[3]))}

            plan_m = pr.Plan([pm], pr.PR_MODE_MIXED)
            t_m = timed(lambda: plan_m.solve([um], uT=[uT_mixed], want_log=False), reps=3, warm=1)
            del plan_m
            torch.cuda.empty_cache()
            plan_p = pr.Plan([pm], pr.PR_MODE_FP64 | pr.PR_MODE_PER_SLICE)
            t_p = timed(lambda: plan_p.solve([um], uT=[uT_plain], want_log=False), reps=3, warm=1)
            del plan_p
            torch.cuda.empty_cache()
            extra["mixed_vs_plain_fp64"] = {
                "workload": "%s: %dx%dx%d, P=%d, K=%d, %d fine / %d coarse steps" % (
                    args.mixed_config, pm.n[0], pm.n[1], pm.n[2], pm.P, pm.K, pm.nt_fine, pm.nt_coarse),
                "batched_fp32_sweeps_ms": round(t_m, 2), "plain_fp64_per_slice_ms": round(t_p, 2),
                "speedup": round(t_p / t_m, 3),
                "error_vs_fp64_serial_fine": {"batched_fp32_sweeps": errs(uT_mixed, u_fine64),
                                              "plain_fp64_per_slice": errs(uT_plain, u_fine64)},
                "batched_fp32_vs_plain_fp64_parareal": errs(uT_mixed, uT_plain)}
            del um, u_fine64, uT_mixed, uT_plain
            torch.cuda.empty_cache()
            log("mixed comparison", extra["mixed_vs_plain_fp64"])

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(p, u0_np)
        log("cpu baseline", cpu)

    line = {
        "metric": "fine-sweep GLUP/s + % peak HBM GB/s; Parareal time-to-solution vs plain FP64",
        "value": round(value, 3),
        "unit": "GLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": "%s: %dx%dx%d periodic advection-diffusion, P=%d slices, K=%d, %d fine RK4 / %d "
                               "coarse Euler steps, %s" % (args.config, p.n[0], p.n[1], p.n[2], p.P, p.K,
                                                           p.nt_fine, p.nt_coarse,
                                                           "FP32 sweeps + FP64 correction" if mixed else "FP64"),
                   "grid": list(p.n), "P": p.P, "K": p.K, "nt_fine": p.nt_fine, "nt_coarse": p.nt_coarse},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "achievable": ceiling["gbs"], "frac_of_achievable": round(achieved / ceiling["gbs"], 4),
                     "achievable_probe": ceiling,
                     "kernel": "%s (%s)" % (kernel_of(fine_variant), fine_variant), "coarse_kernel": coarse_variant,
                     "avg_launch_us": round(avg_launch_s * 1e6, 2),
                     "algorithmic_bytes_per_launch": int(bytes_per_launch)},
        "cpu_baseline": cpu,
        "defect_dk": [float("%.3e" % d) for d in dk],
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
