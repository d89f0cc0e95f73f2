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
import re
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

# HBM bytes per batched fused-RK4 launch from rocprofv3 FETCH_SIZE /
# WRITE_SIZE (scaled by the plain-copy calibration), recorded with the
# SHA-256 of the kernel source they were taken on.  A figure is reported only
# while the source is unchanged and the plan still launches that variant.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1409_8563_amd", "csrc", "stencil_kernels.hip")


def measured_traffic(variant, workload):
    """(bytes per launch or None, note)."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None, "no recorded counters"
    with open(KERNEL_SOURCE, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if rec.get("stencil_kernels_sha256") != sha:
        return None, "kernel source changed since the counters were taken"
    v = rec.get("per_launch_bytes", {}).get("%s@%s" % (variant, workload))
    if v is None:
        return None, "no counters for this variant and workload"
    return int(v), "rocprofv3 FETCH_SIZE + WRITE_SIZE, %s" % rec.get("summary", "profiles/")


def kernel_of(variant):
    """HIP kernel that a fine variant launches."""
    if variant == "rk4_unfused_reference":
        return "rk4_stage_ref"
    for prefix, kernel in (("rk4w_", "rk4_step_rows"), ("rk4s_", "rk4_step_rows"), ("rk4x_", "rk4_step_rows"),
                           ("rk4b_", "rk4_step_fused1b"), ("rk4h_", "rk4_half_rows"), ("rk4hx_", "rk4_half_rows"),
                           ("rk4r_", "rk4_step_fused1r"),
                           ("rk4_", "rk4_step_fused")):
        if variant.startswith(prefix):
            return kernel
    return "rk4_stage_ref"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


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
        tr, _ = measured_traffic(fv, name)
        out[name] = {"glups": round(lups / ms / 1e6, 1), "gbs": round(lups * 2 * es / ms / 1e6, 1),
                     "frac": round(lups * 2 * es / ms / 1e6 / HBM_PEAK_GBS, 4),
                     "launch_us": round(ms * 1e3, 1), "kernel": "%s (%s)" % (kernel_of(fv), fv),
                     "traffic": tr, "traffic_over_algorithmic": None if tr is None else round(tr / (lups * 2 * es), 3)}
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
    tr, _ = measured_traffic(fv, "paper_setup_order4_fp64")
    out["paper_setup_order4_fp64"] = {"glups": round(lups / ms / 1e6, 1), "gbs": round(lups * 16 / ms / 1e6, 1),
                                      "frac": round(lups * 16 / ms / 1e6 / HBM_PEAK_GBS, 4),
                                      "launch_us": round(ms * 1e3, 1), "kernel": "%s (%s)" % (kernel_of(fv), fv),
                                      "traffic": tr,
                                      "traffic_over_algorithmic": None if tr is None else round(tr / (lups * 16), 3)}
    del u, o
    torch.cuda.empty_cache()
    insts = W.batched_config(64)
    probs = [W.Problem(**{**q.__dict__, "K": 1}) for q, _ in insts]
    u0s = [torch.randn(tuple(reversed(q.n)), dtype=torch.float64, device="cuda") for q in probs]
    # the workload's own configuration is the autotuned plan; the built-in
    # kernel choice is reported beside it
    lups = sum(q.P * q.npts * q.nf for q in probs)
    rates = {}
    for label in ("builtin", "tuned"):
        plan = pr.Plan(probs, pr.PR_MODE_MIXED | pr.PR_MODE_TIMED)
        if label == "tuned":
            t0 = time.perf_counter()
            plan.autotune()
            tune_s = time.perf_counter() - t0
        plan.solve(u0s, want_log=False)
        best = float("inf")
        for _ in range(3):
            plan.solve(u0s, want_log=False)
            best = min(best, plan.timings()["fine_ms"])
        rates[label] = (best, plan)
    fine_ms, plan = rates["tuned"]
    # whole-row variants name their row width; each group of the workload is one grid size
    grid_of = {v: int(re.search(r"_x(\d+)_", v).group(1)) for v, _, _ in plan.fine_groups()
               if re.search(r"_x(\d+)_", v)}
    out["c4_batched_64"] = {"glups": round(lups / fine_ms / 1e6, 1),
                            "gbs": round(lups * 8 / fine_ms / 1e6, 1),
                            "frac": round(lups * 8 / fine_ms / 1e6 / HBM_PEAK_GBS, 4),
                            "tuned": True, "tuning_s": round(tune_s, 2),
                            "glups_builtin_choice": round(lups / rates["builtin"][0] / 1e6, 1),
                            "kernel": "%s (%s)" % (kernel_of(plan.kernel_variants()[0]), plan.kernel_variants()[0]),
                            "launch_groups": [{"variant": v, "blocks_per_cu": b, "instances": n,
                                               "traffic_per_step": measured_traffic(
                                                   v, "c4_batched_64:%d^3 group" % grid_of[v])[0]
                                               if v in grid_of else None}
                                              for v, b, n in plan.fine_groups()]}
    del rates, plan, u0s
    torch.cuda.empty_cache()
    return out


def workload_solves(pr, W, torch, quick=False):
    """Time-to-solution of every workload on the GPU: batched Parareal (FP32
    sweeps for the mixed workloads, FP64 otherwise; replayed from a recorded
    graph, median of 10 calls after 3, except 512^3: eager, one call after
    one), the pipelined schedule for 128^3 and 256^3, plain per-slice FP64
    Parareal (one F launch per slice and step) and the serial FP64 fine
    sweep (median of `reps` calls after one); and every form's result over
    the whole field for the accuracy check against the FP64 reference
    computed in the CPU leg (for 256^3 also the FP32-sweep iterate after
    each iteration)."""
    import numpy as np

    def timed(fn, reps, warm=1):
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

    out = {}
    names = ["c1_32_fp64", "c2_128_fp64", "c3_256_mixed"] + ([] if quick else ["c5_512_mixed"])
    for name in names:
        p, modes = W.config(name)
        mixed = W.MIXED[name]
        reps = 1 if name == "c5_512_mixed" else (3 if name == "c3_256_mixed" else 5)
        u0 = torch.from_numpy(W.synth_u0(p.n, modes)).cuda()

        def grab(u):
            return u.view(-1).cpu().numpy()   # the whole field

        rec = {"forms": {}}
        uT = torch.empty_like(u0)
        mode = pr.PR_MODE_MIXED if mixed else pr.PR_MODE_FP64
        big = name == "c5_512_mixed"
        # the batched solve replayed from a recorded graph, median of 10 after 3 warm calls (the
        # 512^3 workload: eager, one call after one warm call); plan creation (workspace allocation,
        # tables) and the first call (which records the graph) are timed on their own
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = pr.Plan([p], mode | (0 if big else pr.PR_MODE_GRAPH))
        torch.cuda.synchronize()
        t_create = (time.perf_counter() - t0) * 1e3
        t0 = time.perf_counter()
        plan.solve([u0], uT=[uT], want_log=False)
        torch.cuda.synchronize()
        t_first = (time.perf_counter() - t0) * 1e3
        t = timed(lambda: plan.solve([u0], uT=[uT], want_log=False), 1 if big else 10, 1 if big else 3)
        batched = grab(uT)
        rec["forms"]["parareal_batched_" + ("fp32_sweeps" if mixed else "fp64")] = {
            "ms": round(t, 3), "result": batched, "plan_create_ms": round(t_create, 1),
            "first_call_ms": round(t_first, 1),
            "note": "eager launches" if big else "replayed from a recorded HIP graph; the first call records it"}
        del plan
        torch.cuda.empty_cache()
        if name == "c3_256_mixed":
            # the FP32-sweep iterate after every iteration k (a solve stopped after k corrections
            # computes the same iterate as the k-th of the full solve), for its error against the
            # FP64 reference per iteration
            its = {}
            for k in range(1, p.K):
                pk, _ = W.config(name, K=k)
                plan = pr.Plan([pk], mode)
                plan.solve([u0], uT=[uT], want_log=False)
                its[k] = grab(uT)
                del plan
                torch.cuda.empty_cache()
            its[p.K] = batched
            rec["per_iteration"] = its
        if name in ("c2_128_fp64", "c3_256_mixed"):
            # the pipelined schedule (Section 2.2.1) in two slice groups
            plan = pr.Plan([p], mode | pr.PR_MODE_PIPELINED | pr.PR_MODE_PIPELINE_GROUPS(2))
            t = timed(lambda: plan.solve([u0], uT=[uT], want_log=False), reps)
            res = grab(uT)
            rec["forms"]["parareal_batched_pipelined"] = {
                "ms": round(t, 3), "result": res, "slice_groups": 2,
                "bitwise_equal_to_batched": bool(np.array_equal(res, batched))}
            del plan
            torch.cuda.empty_cache()
        plan = pr.Plan([p], pr.PR_MODE_FP64 | pr.PR_MODE_PER_SLICE)
        t = timed(lambda: plan.solve([u0], uT=[uT], want_log=False), reps)
        rec["forms"]["parareal_plain_fp64_per_slice"] = {"ms": round(t, 3), "result": grab(uT)}
        del plan
        torch.cuda.empty_cache()
        t = timed(lambda: pr.fine_sweep(p, u0, 0, p.nt_fine, u_out=uT), reps)
        rec["forms"]["serial_fine_fp64"] = {"ms": round(t, 3), "result": grab(uT)}
        out[name] = rec
        del u0, uT
        torch.cuda.empty_cache()
        log("solved", name, {k: v["ms"] for k, v in rec["forms"].items()})

    # the 64 uneven instances: one plan over all of them
    insts = W.batched_config(64)
    probs = [q for q, _ in insts]
    u0s = [torch.from_numpy(W.synth_u0(q.n, m)).cuda() for q, m in insts]
    uTs = [torch.empty_like(u) for u in u0s]
    def grab_all():
        return [u.view(-1).cpu().numpy() for u in uTs]

    rec = {"forms": {}}
    plan = pr.Plan(probs, pr.PR_MODE_MIXED | pr.PR_MODE_GRAPH)
    plan.autotune()
    t = timed(lambda: plan.solve(u0s, uT=uTs, want_log=False), 3)
    rec["forms"]["parareal_batched_fp32_sweeps"] = {"ms": round(t, 3), "result": grab_all(),
                                                    "note": "autotuned plan, replayed from a recorded HIP graph"}
    del plan
    torch.cuda.empty_cache()
    plan = pr.Plan(probs, pr.PR_MODE_FP64 | pr.PR_MODE_PER_SLICE)
    t = timed(lambda: plan.solve(u0s, uT=uTs, want_log=False), 1)
    rec["forms"]["parareal_plain_fp64_per_slice"] = {"ms": round(t, 3), "result": grab_all()}
    del plan
    torch.cuda.empty_cache()

    def serial_all():
        for q, u, o in zip(probs, u0s, uTs):
            pr.fine_sweep(q, u, 0, q.nt_fine, u_out=o)
    t = timed(serial_all, 1)
    rec["forms"]["serial_fine_fp64"] = {"ms": round(t, 3), "result": grab_all(),
                                        "note": "the 64 instances one after another on one stream"}
    out["c4_batched_64"] = rec
    log("solved c4_batched_64", {k: v["ms"] for k, v in rec["forms"].items()})
    del u0s, uTs
    torch.cuda.empty_cache()
    return out


def lscpu_summary():
    """Model, sockets, cores and threads of the host (lscpu), for the CPU leg."""
    import subprocess
    info = {}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except (OSError, subprocess.SubprocessError):
        return {"lscpu": "unavailable"}
    for line in txt.splitlines():
        k, _, v = line.partition(":")
        k = k.strip()
        if k in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)", "L3 cache",
                 "NUMA node(s)"):
            info[k] = v.strip()
    info["usable_threads"] = len(os.sched_getaffinity(0))
    return info


def cpu_leg(p_main, u0_np, solves, budget_s=8.0):
    """The CPU leg: the FP64 oracle timed on this host, and the FP64
    references of the workloads' results.

    * cpu_baseline value: the oracle's RK4 steps on one field of the timed
      workload, on all host threads (bounded sample).
    * per workload: wall time of one oracle fine step and one coarse step on
      1 thread and on 8 threads, and the oracle's Parareal and serial-fine
      wall times extrapolated from them (the 32^3 workload's are measured
      end to end instead).
    * accuracy: max-abs and relative-L2 error of every GPU result against the
      FP64 reference of the same computation: the grid oracle over the full
      field for the 32^3 workload, elsewhere the oracle's per-Fourier-mode
      model of the same discrete scheme (equal to the grid oracle up to
      rounding, pinned by the tests) synthesised over the whole field by an
      inverse FFT."""
    import numpy as np
    import oracle
    from oracle import spectral
    import workloads as W
    oracle.lib()
    all_threads = oracle.threads()

    t = time.perf_counter()
    oracle.fine_steps(p_main, 0, 1, u0_np)
    one = time.perf_counter() - t
    m = int(max(2, min(400, budget_s / max(one, 1e-6))))
    t = time.perf_counter()
    oracle.fine_steps(p_main, 0, m, u0_np)
    dt = time.perf_counter() - t
    base = {"value": m * p_main.npts / dt / 1e9, "unit": "GLUP/s", "cores": all_threads, "kind": "oracle",
            "sample": "%d FP64 RK4 steps of the oracle on one %dx%dx%d field (%.1f s) on %d host threads"
                      % (m, p_main.n[0], p_main.n[1], p_main.n[2], dt, all_threads),
            "host": lscpu_summary()}

    def step_times(p, u, threads):
        oracle.set_threads(threads)
        t0 = time.perf_counter()
        oracle.fine_steps(p, 0, 1, u)
        tf = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.coarse_steps(p, 0, 1, u)
        tc = time.perf_counter() - t0
        return tf, tc

    per = {}
    for name in ("c1_32_fp64", "c2_128_fp64", "c3_256_mixed", "c5_512_mixed"):
        p, modes = W.config(name)
        u0 = W.synth_u0(p.n, modes)
        entry = {}
        for th in (1, 8):
            if name == "c1_32_fp64":
                oracle.set_threads(th)
                t0 = time.perf_counter()
                U, _ = oracle.parareal(p, u0, K=p.K)
                tp = time.perf_counter() - t0
                t0 = time.perf_counter()
                oracle.serial_fine(p, u0)
                ts = time.perf_counter() - t0
                entry["threads_%d" % th] = {"parareal_s": round(tp, 3), "serial_fine_s": round(ts, 3),
                                            "how": "measured end to end"}
                ref = U[-1].ravel()
            else:
                # the 256^3 and 512^3 grids are timed on a slab of 32 z planes
                # (same per-point work) and scaled by n_z / 32
                nzs = min(p.n[2], 32)
                ps = W.Problem(**{**p.__dict__, "n": (p.n[0], p.n[1], nzs)})
                tf, tc = step_times(ps, u0[:nzs] if nzs == p.n[2] else W.synth_u0(ps.n, modes), th)
                tf, tc = tf * p.n[2] / nzs, tc * p.n[2] / nzs
                tp = p.K * p.P * p.nf * tf + (p.K + 1) * p.P * p.nc * tc
                how = ("extrapolated from one timed fine and one timed coarse step%s: K*P*Nf fine + (K+1)*P*Nc "
                       "coarse steps" % ("" if nzs == p.n[2] else
                                        " on a %dx%dx%d slab, scaled by n_z" % (p.n[0], p.n[1], nzs)))
                entry["threads_%d" % th] = {"fine_step_s": round(tf, 4), "coarse_step_s": round(tc, 4),
                                            "parareal_s": round(tp, 1), "serial_fine_s": round(p.nt_fine * tf, 1),
                                            "how": how}
        oracle.set_threads(all_threads)
        if name != "c1_32_fp64" and name in solves:
            sol = spectral.ModalSolution(p, modes)
            ref = sol.iterate_fft(p.K, p.P).ravel()
        entry["reference"] = ("grid oracle, whole field" if name == "c1_32_fp64" else
                              "oracle per-mode model synthesised over the whole field (inverse FFT)")
        if name in solves and ref is not None:
            entry["accuracy_vs_fp64_parareal"] = {
                form: errs(rec["result"], ref) for form, rec in solves[name]["forms"].items()
                if form.startswith("parareal")}
            del ref
            fine_ref = (oracle.serial_fine(p, u0).ravel() if name == "c1_32_fp64" else
                        sol.serial_fine_fft().ravel())
            entry["accuracy_vs_fp64_serial_fine"] = {
                form: errs(rec["result"], fine_ref) for form, rec in solves[name]["forms"].items()}
            if "per_iteration" in solves[name]:
                entry["per_iteration_vs_fp64"] = [
                    {"k": k, "vs_fp64_parareal": errs(res, sol.iterate_fft(k, p.P).ravel()),
                     "vs_fp64_serial_fine": errs(res, fine_ref)}
                    for k, res in sorted(solves[name]["per_iteration"].items())]
            del fine_ref
        per[name] = entry
        log("cpu leg", name, entry)
    if "c4_batched_64" in solves:
        insts = W.batched_config(64)
        rec = solves["c4_batched_64"]
        worst = {}
        worst_fine = {}
        for i, (q, modes) in enumerate(insts):
            sol = spectral.ModalSolution(q, modes)
            r = sol.iterate_fft(q.K, q.P).ravel()
            rf = sol.serial_fine_fft().ravel()
            for form, fr in rec["forms"].items():
                for tgt, rr in ((worst, r), (worst_fine, rf)):
                    if tgt is worst and not form.startswith("parareal"):
                        continue
                    e = errs(fr["result"][i], rr)
                    w = tgt.setdefault(form, {"max_abs": 0.0, "rel_l2": 0.0})
                    w["max_abs"] = max(w["max_abs"], e["max_abs"])
                    w["rel_l2"] = max(w["rel_l2"], e["rel_l2"])
        sizes = sorted({q.n[0] for q, _ in insts})
        c4 = {"reference": "oracle per-mode model per instance over its whole field (inverse FFT); worst instance",
              "accuracy_vs_fp64_parareal": worst, "accuracy_vs_fp64_serial_fine": worst_fine}
        for th in (1, 8):
            tot_p = tot_s = 0.0
            cache = {}
            for q, modes in insts:
                if q.n[0] not in cache:
                    cache[q.n[0]] = step_times(q, W.synth_u0(q.n, modes), th)
                tf, tc = cache[q.n[0]]
                tot_p += q.K * q.P * q.nf * tf + (q.K + 1) * q.P * q.nc * tc
                tot_s += q.nt_fine * tf
            c4["threads_%d" % th] = {"parareal_s": round(tot_p, 1), "serial_fine_s": round(tot_s, 1),
                                     "how": "extrapolated per instance from one timed fine and coarse step of "
                                            "each grid size %s" % sizes}
        oracle.set_threads(all_threads)
        per["c4_batched_64"] = c4
        log("cpu leg c4", c4)
    base["per_workload"] = per
    return base


def errs(x, r):
    import numpy as np
    x = np.asarray(x, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    d = x - r
    return {"max_abs": float("%.3e" % np.max(np.abs(d))),
            "rel_l2": float("%.3e" % np.sqrt(np.sum(d * d) / np.sum(r * r)))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2_128_fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--no-solves", action="store_true",
                    help="skip the per-workload time-to-solution and accuracy section")
    ap.add_argument("--quick", action="store_true", help="leave the 512^3 workload out of that section")
    ap.add_argument("--no-per-config", action="store_true",
                    help="skip the per-workload F kernel rates (all five workloads)")
    ap.add_argument("--schedules", action="store_true",
                    help="only run the workload's solve in the phase-by-phase and the pipelined schedule "
                         "(two calls each, for a kernel trace) and exit")
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
    if args.schedules:
        uT = torch.empty_like(u0)
        for name, extra in (("phase-by-phase", 0),
                            ("pipelined, 2 slice groups", pr.PR_MODE_PIPELINED | pr.PR_MODE_PIPELINE_GROUPS(2))):
            sp = pr.Plan([p], mode | extra)
            for rep in range(2):
                torch.cuda.synchronize()
                t = time.perf_counter()
                sp.solve([u0], uT=[uT], want_log=False)
                torch.cuda.synchronize()
                log("%s solve %d: %.2f ms" % (name, rep, (time.perf_counter() - t) * 1e3))
            del sp
        return
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
    traffic, traffic_note = measured_traffic(fine_variant, args.config)
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
    solves = {}
    if not args.no_solves:
        solves = workload_solves(pr, W, torch, quick=args.quick)
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu leg (oracle) ...")
        cpu = cpu_leg(p, u0_np, solves)
        log("cpu baseline", {k: v for k, v in cpu.items() if k != "per_workload"})
    if solves:
        wl = {}
        for name, rec in solves.items():
            e = {"time_to_solution_ms": {form: r["ms"] for form, r in rec["forms"].items()}}
            for form, r in rec["forms"].items():
                extra_t = {k: r[k] for k in ("plan_create_ms", "first_call_ms", "note") if k in r}
                if extra_t:
                    e.setdefault("time_to_solution_notes", {})[form] = extra_t
            pf = rec["forms"].get("parareal_batched_pipelined")
            if pf is not None:
                e["pipelined"] = {"slice_groups": pf["slice_groups"],
                                  "bitwise_equal_to_batched": pf["bitwise_equal_to_batched"]}
            if cpu is not None and name in cpu["per_workload"]:
                c = cpu["per_workload"][name]
                for key in ("reference", "accuracy_vs_fp64_parareal", "accuracy_vs_fp64_serial_fine",
                            "per_iteration_vs_fp64"):
                    if key in c:
                        e[key] = c[key]
                e["oracle_wall_s"] = {k: v for k, v in c.items() if k.startswith("threads_")}
            wl[name] = e
        extra["workloads"] = wl
    if cpu is not None:
        cpu.pop("per_workload", None)

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
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_source": traffic_note,
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
