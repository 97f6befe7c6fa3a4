#!/usr/bin/env python3
"""Benchmark: CTD time steps per second for 3D Allen-Cahn at 1024 nodes per axis.

One "step" is one time step of the stabilized semi-implicit scheme solved in
separated form by the HIP library (greedy enrichment, alternating fixed-point
sweeps, banded 1D solves, cubic contractions, energy on the separated
quadrature), on seeded synthetic cosine initial data held on the GPU.  The
fixed-point iteration of mode m starts from mode m of u^k (`--init warm`,
the default; the paper leaves the initial guess open) or from the
counter-based random vector (`--init hash`); every leg uses the same choice,
and leg 9 reports the other one.

Legs (rank 0, one GPU):
  1. mixed precision (FP32 MFMA contractions, FP64 solves/decisions), adaptive:
     W warmup steps, then K timed steps bracketed by device synchronisation;
     per-kernel HIP-event timing inside the library gives the roofline of
     the dominant kernel.
  2. plain FP64, adaptive: same protocol (context: the mixed path must beat it).
  3. accuracy (relative nodal l2, the paper's error metric): (a) one mixed
     step from the FP64 state u^k with the FP64 step's decisions, against the
     FP64 step; (b) the mixed run after all its steps against an FP64 replay of
     its decisions; (c) for scale, FP64 against FP64 started from u0 with
     amplitudes perturbed by 1e-14 (same decisions): the capped greedy
     decomposition amplifies any difference from step to step.
     (d) the same for a single step: FP64 from the FP64 u^k with amplitudes
     perturbed by 1e-14, same decisions.
  4. CPU baseline: the oracle (numpy/scipy FP64) timed on a bounded sample of
     the same workload on the host cores.
  5. batched sample: uneven 2D instances from the batched workload's generator
     stepped concurrently by ctd_batch_step (worker streams), against one
     worker; reported as instance-steps/s.
  6. served sample: a Poisson request stream from the served workload's
     generator (request count and step counts scaled down, sizes and rate as
     generated) through ctd_server_*; p50/p99 latency from arrival to
     completion and aggregate steps/s.
  7. (p, s) sweep: set-up time and step cost of the 256^3 workload at the
     CFE parameters (1, 1), (1, 2), (2, 2), (3, 3) (band half-widths 3, 5, 7).
  8. adaptive full-solve fallback (2D): full CFE steps of a 1024^2 instance
     (the second from a field state), step time and the FP64 MFMA rate of the
     dense eigenbasis products.
  9. the other initial guess: the headline workload and protocol with the
     counter-based initial vector of a mode (the headline uses mode m of u^k,
     `--init`), steps/s, sweeps, and one mixed step against FP64 with the
     same decisions.
Prints ONE JSON line on stdout; progress goes to stderr.  `--only LEG`
(actd, batched, served, ps) runs a single leg and prints its JSON instead,
for profiling that leg alone; it is not the benchmark line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32_mfma": 157.3e12, "fp64_mfma": 78.6e12, "hbm": 8.0e12}
# HBM traffic per launch measured with rocprofv3 counters on this workload
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "ctd_step_ac3d_n1024_mixed_hbm_traffic.md")
# kernel [grid work-items] of each class at the timed shape (M_k = 128)
KERNEL_NAMES = {"cubic_g": "k_cubic_g32 [245760]", "cubic_h": "k_cubic_h32 [512000]",
                "cubic_gred": "k_cubic_gred32 [491520]"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_leg(ctd, inst, precision, warmup, steps, decisions=None, profile=True, init="warm",
            warm_infos=None):
    """W warmup steps (the last one timed per kernel class, all classes), then
    K timed steps with HIP events around the launches of the dominant class
    only (events on every launch would slow the launch cadence)."""
    import torch
    sched = "replay" if decisions is not None else "adaptive"
    s = ctd.Solver(inst, precision=precision, schedule=sched, energy=True, init=init)
    if decisions is not None:
        s.set_decisions(decisions)
    dec = []
    prof_all = {}
    for k in range(warmup):
        last = profile and k == warmup - 1
        if last:
            s.profile(True)
        info = s.step(1)[0]
        dec += s.decisions()
        if warm_infos is not None:
            warm_infos.append(info)
        if last:
            prof_all = s.profile_read()
            s.profile(False)
        log(f"  [{precision}/{sched}] warmup {k}: {info['ms']:.0f} ms modes={info['modes']} "
            f"sweeps={info['sweeps']}")
    if profile:
        dom = max(prof_all.items(), key=lambda kv: kv[1]["ms"])[0] if prof_all else None
        s.profile(True, classes=[dom] if dom else None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for k in range(steps):
        info = s.step(1)[0]
        dec += s.decisions()
        infos.append(info)
        log(f"  [{precision}/{sched}] step {k}: {info['ms']:.0f} ms modes={info['modes']} "
            f"sweeps={info['sweeps']} E={info['energy']:.9e}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = s.profile_read() if profile else {}
    if profile:
        s.profile(False)
    return s, infos, t1 - t0, {"timed": prof, "warmup": prof_all}, dec


def traffic_of(name, precision, workload):
    if workload != "ac3d_n1024" or precision != "mixed":
        return None
    from paper_2410_15519_amd.profsum import traffic_from_summary
    k = KERNEL_NAMES.get(name)
    return traffic_from_summary(TRAFFIC_SUMMARY, k) if k else None


def roofline_of(prof, precision, workload="ac3d_n1024"):
    # dominant kernel = largest summed device time (the only class timed in
    # the timed steps)
    name, v = max(prof.items(), key=lambda kv: kv[1]["ms"])
    avg_ms = v["ms"] / v["launches"]
    traffic = traffic_of(name, precision, workload)
    if name in ("cubic_g", "cubic_h", "energy", "mxy_build"):
        peak = PEAK["fp32_mfma"] if (precision == "mixed" and name != "energy") else PEAK["fp64_mfma"]
        per_launch = v["flops"] / v["launches"]
        achieved = per_launch / (avg_ms * 1e-3)
        return name, {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12,
                      "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
                      "kernel": name, "avg_launch_us": avg_ms * 1e3,
                      "algorithmic_per_launch": per_launch}
    per_launch = v["bytes"] / v["launches"]
    achieved = per_launch / (avg_ms * 1e-3)
    return name, {"bound": "hbm", "achieved": achieved / 1e9, "peak": PEAK["hbm"] / 1e9,
                  "unit": "GB/s", "frac": achieved / PEAK["hbm"], "traffic": traffic,
                  "kernel": name, "avg_launch_us": avg_ms * 1e3,
                  "algorithmic_per_launch": per_launch}


def cpu_baseline(inst, gpu_step0_ms, gpu_sweeps0):
    """The oracle (plain numpy/scipy FP64) on whole time steps of the same
    workload: step 1 from the seeded initial field, as the GPU's first step.
    A step from the 8-mode initial field is the cheapest step of the run
    (M_k = 8 in the cubic contraction); the GPU's time for the same step is
    reported beside it, so the ratio compares like with like."""
    from oracle.ctd import ctd_step, state_from_instance
    from oracle.scheme import problem_from_instance
    try:
        from threadpoolctl import threadpool_info
        cores = max((i.get("num_threads", 1) for i in threadpool_info()), default=os.cpu_count())
    except Exception:
        cores = os.cpu_count()
    pr = problem_from_instance(inst)
    st = state_from_instance(inst)
    t0 = time.perf_counter()
    _, lg = ctd_step(pr, st, 0)
    el = time.perf_counter() - t0
    log(f"  [cpu oracle] whole step 1: {el:.1f} s, {len(lg.iters)} modes, {sum(lg.iters)} sweeps")
    return {"value": 1.0 / el, "unit": "steps/s", "cores": int(cores), "kind": "oracle",
            "sample": (f"one whole oracle time step (step 1 from the seeded {len(inst.amp)}-mode "
                       f"initial field, M_k = {len(inst.amp)}; {len(lg.iters)} modes, "
                       f"{sum(lg.iters)} sweeps, {el:.1f} s) of the {inst.nodes[0]}^{inst.dim} "
                       f"workload; later steps (M_k = {inst.max_modes}) cost more on both sides"),
            "gpu_same_step_steps_per_s": 1e3 / gpu_step0_ms if gpu_step0_ms else None,
            "gpu_same_step_sweeps": gpu_sweeps0}


def rel_l2(a, b):
    import numpy as np
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def ac2d_leg(ctd, steps=50, check_steps=3):
    """The 2D 128^2 workload (eps 0.02, dt 1e-3, 4 cosine modes, cap 64), FP64:
    steps/s over its 50 steps (adaptive), and the GPU against the CPU oracle
    (relative nodal l2) after each of the first steps with the oracle's
    decisions replayed."""
    import torch
    from oracle.ctd import ctd_step, full_field, state_from_instance
    from oracle.scheme import problem_from_instance
    from workloads import make_instance
    inst = make_instance("ac2d_n128")
    s = ctd.Solver(inst, precision="fp64", energy=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = s.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    s.close()
    pr = problem_from_instance(inst)
    st = state_from_instance(inst)
    refs, logs = [], []
    for k in range(check_steps):
        st, lg = ctd_step(pr, st, k)
        refs.append(full_field(st))
        logs.append(lg.iters)
    errs = []
    with ctd.Solver(inst, precision="fp64", schedule="replay") as r:
        r.set_decisions(logs)
        for k in range(check_steps):
            r.step(1)
            errs.append(rel_l2(r.reconstruct(), refs[k]))
    out = {"workload": "ac2d_n128", "precision": "fp64", "steps": steps, "steps_per_s": steps / el,
           "ms_per_step": 1e3 * el / steps,
           "modes_per_step": sum(i["modes"] for i in infos) / steps,
           "sweeps_per_step": sum(i["sweeps"] for i in infos) / steps,
           "energy_first_last": [infos[0]["energy"], infos[-1]["energy"]],
           "energy_increases": int(sum(i["energy_increase"] for i in infos)),
           "rel_l2_vs_oracle_first_steps": errs}
    log(f"  [ac2d_n128] {out['steps_per_s']:.1f} steps/s FP64, vs oracle {errs}")
    return out


def ac3d_n256_leg(ctd, steps=100):
    """The 3D 256^3 workload (eps 0.01, dt 5e-4, 8 cosine modes, cap 64):
    steps/s of its 100 steps in mixed precision and in FP64 (adaptive), the
    mixed run against an FP64 replay of its decisions after all steps and for
    its last step alone (from the FP64 state), and the first step of both
    paths against the CPU oracle replaying the oracle's decisions."""
    import numpy as np
    import torch
    from oracle.ctd import ctd_step, full_field, state_from_instance
    from oracle.scheme import problem_from_instance
    from workloads import Instance, make_instance
    inst = make_instance("ac3d_n256")
    out = {"workload": "ac3d_n256", "steps": steps}
    dec = {}
    for prec in ("mixed", "fp64"):
        s = ctd.Solver(inst, precision=prec, energy=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = s.step(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        dec[prec] = s.decisions()
        if prec == "mixed":
            Umix = s.reconstruct()
        s.close()
        out[prec] = {"steps_per_s": steps / el, "ms_per_step": 1e3 * el / steps,
                     "sweeps_per_step": sum(i["sweeps"] for i in infos) / steps,
                     "modes_per_step": sum(i["modes"] for i in infos) / steps,
                     "energy_increases": int(sum(i["energy_increase"] for i in infos))}
        log(f"  [ac3d_n256] {prec}: {out[prec]['steps_per_s']:.2f} steps/s, "
            f"{out[prec]['sweeps_per_step']:.0f} sweeps/step")
    # FP64 replay of the mixed decisions: accumulated and last-step differences
    r = ctd.Solver(inst, precision="fp64", schedule="replay")
    r.set_decisions(dec["mixed"][:-1])
    r.step(steps - 1)
    amp, fac = r.modes()
    k_prev = r.step_index
    r.set_decisions(dec["mixed"][-1:])
    r.step(1)
    U64 = r.reconstruct()
    r.close()
    out["rel_l2_accum_mixed_vs_fp64"] = rel_l2(Umix, U64)
    st = Instance(**{**inst.__dict__, "amp": amp, "factors": fac})
    one = ctd.Solver(st, precision="mixed", schedule="replay")
    one.step_index = k_prev
    one.set_decisions(dec["mixed"][-1:])
    one.step(1)
    out["rel_l2_last_step_mixed_vs_fp64"] = rel_l2(one.reconstruct(), U64)
    one.close()
    # first step against the oracle (its decisions replayed on the GPU)
    pr = problem_from_instance(inst)
    t0 = time.perf_counter()
    st1, lg = ctd_step(pr, state_from_instance(inst), 0)
    t_or = time.perf_counter() - t0
    ref = full_field(st1)
    for prec in ("fp64", "mixed"):
        with ctd.Solver(inst, precision=prec, schedule="replay") as g:
            g.set_decisions([lg.iters])
            g.step(1)
            out[f"rel_l2_step1_{prec}_vs_oracle"] = rel_l2(g.reconstruct(), ref)
    out["oracle_step1_s"] = t_or
    log(f"  [ac3d_n256] mixed vs fp64: accumulated {out['rel_l2_accum_mixed_vs_fp64']:.2e}, "
        f"last step {out['rel_l2_last_step_mixed_vs_fp64']:.2e}; step 1 vs oracle "
        f"fp64 {out['rel_l2_step1_fp64_vs_oracle']:.2e} mixed {out['rel_l2_step1_mixed_vs_oracle']:.2e}")
    return out


def batched_leg(ctd, count=512, steps=2, workers=8, init="warm", sample=(0, 255, 511),
                executors=("lockstep", "streams")):
    """Instance-steps/s of the uneven 2D batch (the batch2d_512 instances)
    under both executors: lockstep rounds of multi-instance launches, and
    the pool of worker streams.  Sampled instances of the lockstep run are
    compared with the standalone solver bitwise."""
    import numpy as np
    import torch
    from workloads import make_batch
    insts = make_batch(count=count)
    out = {"instances": count, "steps": steps, "precision": "mixed",
           "nodes_min": min(int(i.nodes[0]) for i in insts),
           "nodes_max": max(int(i.nodes[0]) for i in insts)}
    kept = {}
    for ex in executors:
        b = ctd.Batch(insts, precision="mixed", init=init)
        b.set_mode(ex)
        b.set_workers(workers)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = b.step(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        if ex == "lockstep":
            kept = {i: b.modes(i) for i in sample if i < count}
        b.close()
        out[f"instance_steps_per_s_{ex}"] = count * steps / el
        out[f"s_{ex}"] = el
        out[f"sweeps_{ex}"] = int(sum(r["sweeps"] for inf in infos for r in inf))
        log(f"  [batched] {count} instances x {steps} steps, {ex}: {el:.2f} s")
    same = True
    for i, (amp, fac) in kept.items():
        with ctd.Solver(insts[i], precision="mixed", init=init) as s:
            s.step(steps)
            ra, rf = s.modes()
        same = same and np.array_equal(amp, ra) and all(np.array_equal(x, y) for x, y in zip(fac, rf))
    out["sampled_equal_standalone"] = bool(same) if kept else None
    return out


def ps_sweep_leg(ctd, workload="ac3d_n256", warmup=1, steps=1, init="warm"):
    """Cost of the CTD step across the CFE parameters (p, s) of the paper's
    Sec. 4 study, on one 3D workload: set-up time (host CFE tables, banded
    matrices, eigenvectors of the fast diagonalisation), ms per step and per
    directional solve after one warm-up step (mixed precision, adaptive)."""
    import torch
    from workloads import make_instance
    out = {"workload": workload, "warmup": warmup, "steps": steps, "cases": []}
    for p, s in ((1, 1), (1, 2), (2, 2), (3, 3)):
        inst = make_instance(workload, patch_s=s, poly_p=p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sv = ctd.Solver(inst, precision="mixed", init=init)
        torch.cuda.synchronize()
        t_init = time.perf_counter() - t0
        sv.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = sv.step(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        sv.close()
        sweeps = sum(i["sweeps"] for i in infos)
        case = {"p": p, "s": s, "band": 2 * s + 1, "init_ms": 1e3 * t_init,
                "ms_per_step": 1e3 * el / steps, "sweeps_per_step": sweeps / steps,
                "modes": int(infos[-1]["modes"]),
                "us_per_directional_solve": 1e6 * el / max(1, sweeps * inst.dim)}
        out["cases"].append(case)
        log(f"  [ps] (p,s)=({p},{s}): init {case['init_ms']:.0f} ms, "
            f"{case['ms_per_step']:.0f} ms/step, {sweeps} sweeps, "
            f"{case['us_per_directional_solve']:.1f} us per directional solve")
    return out


def actd_leg(ctd, n=1024, steps=2):
    """Full-solve fallback of the adaptive algorithm (2D, Sec. 3.3): a 2D
    instance on n x n nodes replaying full CFE steps; the second one starts
    from a field state (one mode per node).  Reports the step time and the
    per-class kernel times, with the FP64 MFMA rate of the full solve's dense
    products (5 products of 2 n^3 flops per step)."""
    import torch
    from workloads import make_instance
    inst = make_instance("ac2d_n128", nodes=n)
    t0 = time.perf_counter()
    sv = ctd.Solver(inst, precision="fp64", schedule="replay", actd=True)
    t_init = time.perf_counter() - t0
    sv.set_decisions(["full"] * steps)
    ms = []
    prof = {}
    for k in range(steps):
        if k == steps - 1:
            sv.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sv.step(1)
        torch.cuda.synchronize()
        ms.append(1e3 * (time.perf_counter() - t0))
    prof = sv.profile_read()
    sv.profile(False)
    sv.close()
    fs = prof.get("full_solve", {})
    out = {"nodes": [n, n], "init_ms": 1e3 * t_init, "ms_per_full_step": ms,
           "classes_ms_last_step": {k: v["ms"] for k, v in prof.items()}}
    if fs:
        out["full_solve_tflops"] = fs["flops"] / (fs["ms"] * 1e-3) / 1e12
        out["full_solve_frac_fp64_mfma"] = out["full_solve_tflops"] * 1e12 / PEAK["fp64_mfma"]
    log(f"  [actd] {n}^2 full steps: {', '.join(f'{x:.1f}' for x in ms)} ms; "
        f"full solve {fs.get('ms', 0):.2f} ms ({out.get('full_solve_tflops', 0):.1f} TFLOP/s); "
        f"classes {({k: round(v, 2) for k, v in out['classes_ms_last_step'].items()})}")
    return out


def mxy_alternatives_leg(ctd, n=1024, steps=5, rd_tol=1e-2, w_rank=8, w_iters=30):
    """The alternatives to the full 2D M_xy integral (Sec. 3.3): the 2D
    workload on n x n nodes stepped (FP64, adaptive) with the full integral,
    with the reduced domain (eq. MxyRD, rd_tol) and with the separated w
    (eq. MxySep, w_rank terms of w_iters updates).  Reports each route's M_xy
    build time per step, the share of elements the reduced domain leaves
    out, the separated route's HBM rate over its row-by-row products (each
    update reads W or W^T once: 2 w_rank w_iters n_q^2 8 bytes per build), and
    the relative nodal l2 difference of each final field from the full one."""
    import torch
    from workloads import make_instance
    inst = make_instance("ac2d_n128", nodes=n)
    nq = 5 * (n - 1)
    routes = {"full": {}, "reduced": {"rd_tol": rd_tol}, "separated": {"w_rank": w_rank, "w_iters": w_iters}}
    out = {"nodes": [n, n], "steps": steps}
    fields = {}
    for name, kw in routes.items():
        with ctd.Solver(inst, precision="fp64", **kw) as sv:
            sv.profile(True, classes=["mxy_build"])
            excl, infos = [], []
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                infos += sv.step(1)
                excl.append(sv.reduced_domain_excluded())
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            prof = sv.profile_read()
            sv.profile(False)
            fields[name] = sv.reconstruct()
        mx = prof.get("mxy_build", {})
        per = mx.get("ms", 0.0) / max(1, mx.get("launches", 1))
        r = dict(kw, ms_per_step=1e3 * el / steps, mxy_build_ms=per,
                 modes_per_step=[i["modes"] for i in infos], sweeps_per_step=[i["sweeps"] for i in infos])
        if name == "reduced":
            r["excluded_share"] = [c / float((n - 1) ** 2) for c in excl]
        if name == "separated":
            r["update_GB_per_s"] = 2 * w_rank * w_iters * nq * nq * 8 / (per * 1e-3) / 1e9
        if name != "full":
            r["rel_l2_vs_full"] = rel_l2(fields[name], fields["full"])
        out[name] = r
    log(f"  [M_xy alternatives] {n}^2: ms/step " + ", ".join(f"{k} {out[k]['ms_per_step']:.1f} "
        f"(modes {out[k]['modes_per_step']}, sweeps {out[k]['sweeps_per_step']})" for k in routes))
    log(f"  [M_xy alternatives] {n}^2: build {out['full']['mxy_build_ms']:.2f} ms full, "
        f"{out['reduced']['mxy_build_ms']:.2f} ms reduced (rd_tol {rd_tol:g}, excluded "
        f"{out['reduced']['excluded_share'][-1]:.3f}, field difference {out['reduced']['rel_l2_vs_full']:.1e}), "
        f"{out['separated']['mxy_build_ms']:.2f} ms separated (rank {w_rank}, {w_iters} updates, "
        f"{out['separated']['update_GB_per_s']:.0f} GB/s, field difference {out['separated']['rel_l2_vs_full']:.1e})")
    return out


def init_leg(ctd, inst, warmup, steps, init):
    """The same workload and protocol as the headline with another initial
    guess of a mode ("hash": the counter-based random vector; "warm": mode m
    of u^k; the paper leaves the initial guess open): steps/s and sweeps, and
    one mixed step against the FP64 step with the same decisions from the same
    FP64 state (relative nodal l2)."""
    import numpy as np
    import torch
    from workloads import Instance
    s, infos, el, _, dec = run_leg(ctd, inst, "mixed", warmup, steps, profile=False, init=init)
    s.close()
    out = {"init": init, "steps_per_s": steps / el, "ms_per_step": 1e3 * el / steps,
           "sweeps_per_step": float(np.mean([i["sweeps"] for i in infos])),
           "modes_per_step": float(np.mean([i["modes"] for i in infos]))}
    # FP64 reference state after warmup + steps - 1 steps (replaying the mixed
    # decisions), then one FP64 and one mixed step from it
    k_prev = warmup + steps - 1
    ref = ctd.Solver(inst, precision="fp64", schedule="replay", init=init)
    ref.set_decisions(dec[:k_prev])
    ref.step(k_prev)
    amp, fac = ref.modes()
    ref.set_decisions(dec[k_prev:])
    ref.step(1)
    n = int(np.prod(inst.nodes))
    U64 = torch.empty(n, dtype=torch.float64, device="cuda")
    ref.reconstruct("f64", out=U64)
    ref.close()
    st = Instance(**{**inst.__dict__, "amp": amp, "factors": fac})
    one = ctd.Solver(st, precision="mixed", schedule="replay", init=init)
    one.step_index = k_prev
    one.set_decisions(dec[k_prev:])
    one.step(1)
    U1 = torch.empty(n, dtype=torch.float64, device="cuda")
    one.reconstruct("f64", out=U1)
    one.close()
    out["rel_l2_step_mixed_vs_fp64"] = float(torch.linalg.norm(U1 - U64) / torch.linalg.norm(U64))
    del U1, U64
    torch.cuda.empty_cache()
    log(f"  [init {init}] {out['steps_per_s']:.3f} steps/s, {out['sweeps_per_step']:.0f} sweeps/step, "
        f"mixed vs FP64 step {out['rel_l2_step_mixed_vs_fp64']:.2e}")
    return out


def served_leg(ctd, count=32, step_scale=20, workers=8, init="warm"):
    """Poisson arrivals into the server; latency from arrival to completion."""
    import numpy as np
    from workloads import make_requests, CONFIGS
    cfg = CONFIGS["serve_mix"]
    lo, hi = cfg["steps_range"]
    reqs = make_requests(count=count, steps_range=(max(1, lo // step_scale), max(1, hi // step_scale)))
    srv = ctd.Server(workers=workers)
    t0 = time.perf_counter()
    tickets = []
    for t_arr, inst in reqs:
        dt = t_arr - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        tickets.append((srv.submit(inst, precision="mixed", init=init), inst))
    for t, _ in tickets:
        srv.wait(t)
    st = [srv.status(t) for t, _ in tickets]
    stats = srv.stats()
    for t, _ in tickets:
        srv.fetch(t)
    srv.close()
    lat = np.array([s["t_done_ms"] - s["t_submit_ms"] for s in st])
    steps = sum(s["steps_done"] for s in st)
    span = max(s["t_done_ms"] for s in st) - min(s["t_submit_ms"] for s in st)
    log(f"  [served] {count} requests, {steps} steps in {span / 1e3:.2f} s; "
        f"p50 {np.percentile(lat, 50):.0f} ms p99 {np.percentile(lat, 99):.0f} ms")
    return {"requests": count, "workers": workers, "rate_per_s": cfg["rate"],
            "steps_range": [max(1, lo // step_scale), max(1, hi // step_scale)],
            "p3d": cfg["p3d"], "steps_total": int(steps),
            "latency_ms_p50": float(np.percentile(lat, 50)),
            "latency_ms_p99": float(np.percentile(lat, 99)),
            "steps_per_s": steps / (span / 1e3), "busy_ms": stats["busy_ms"],
            "sample": (f"{count} requests of the served workload's generator, step counts "
                       f"divided by {step_scale}")}


def _serve_stream(ctd, reqs, rate_scale, workers, init, lockstep=True):
    """Submit (arrival time / rate_scale, instance) pairs on their arrival
    times, wait for all (a progress line every 10 s); returns per-request
    statuses, server stats and the wall time of the run."""
    srv = ctd.Server(workers=workers, lockstep=lockstep)
    t0 = time.perf_counter()
    tickets = []
    last = t0
    pending = list(reqs)
    while pending or tickets and srv.stats()["completed"] + srv.stats()["failed"] < len(reqs):
        now = time.perf_counter()
        while pending and pending[0][0] / rate_scale <= now - t0:
            tickets.append(srv.submit(pending.pop(0)[1], precision="mixed", init=init))
        if now - last >= 10.0:
            st = srv.stats()
            log(f"    [serve] {now - t0:.0f} s: submitted {st['submitted']}, done {st['completed']}, "
                f"running {st['running']}, queued {st['queued']}, steps {st['steps_done']}")
            last = now
        nxt = pending[0][0] / rate_scale - (time.perf_counter() - t0) if pending else 0.05
        time.sleep(min(max(nxt, 0.0005), 0.05))
    for t in tickets:
        srv.wait(t)
    wall = time.perf_counter() - t0
    st = [srv.status(t) for t in tickets]
    stats = srv.stats()
    for t in tickets:
        srv.fetch(t)
    srv.close()
    return st, stats, wall


def served_load_leg(ctd, count=64, workers=8, init="warm", lockstep=True, count70=32):
    """The served workload as generated (Poisson arrivals at 200 req/s, 20 %
    3D with 64-512 nodes per axis, 2D with 64-2048, 20-500 steps per
    request; parameters as the batched workload), its first `count`
    requests: capacity (steps and requests completed per second of busy
    time), p50/p99 latency from arrival to completion at the offered 200
    req/s (the queue grows: the offered load is above capacity), then the
    first `count70` requests offered at 70 % of the measured request
    capacity."""
    import numpy as np
    from workloads import make_requests, CONFIGS
    cfg = CONFIGS["serve_mix"]
    reqs = make_requests(count=count)
    out = {"requests": count, "workers": workers, "offered_rate_per_s": cfg["rate"],
           "lockstep_route": bool(lockstep),
           "steps_total": int(sum(i.steps for _, i in reqs)),
           "p3d": float(np.mean([i.dim == 3 for _, i in reqs]))}
    runs = []
    for label, scale in (("offered", 1.0), ("70pct", None)):
        sub = reqs
        if scale is None:
            cap = runs[0]["requests_per_s_capacity"]
            scale = cfg["rate"] / (0.7 * cap)        # stretch the arrival times
            sub = reqs[:count70]
        # arrival times are divided by rate_scale: 1 = as generated, 1/scale = stretched
        st, stats, wall = _serve_stream(ctd, sub, 1.0 / scale, workers, init, lockstep)
        lat = np.array([x["t_done_ms"] - x["t_submit_ms"] for x in st])
        wait = np.array([x["t_start_ms"] - x["t_submit_ms"] for x in st])
        steps = sum(x["steps_done"] for x in st)
        busy_s = stats["busy_ms"] / 1e3
        r = {"label": label, "requests": len(sub),
             "offered_rate_per_s": cfg["rate"] / scale if label != "offered" else cfg["rate"],
             "wall_s": wall, "busy_s": busy_s, "steps_done": int(steps),
             "steps_per_s_capacity": steps / busy_s, "requests_per_s_capacity": len(sub) / busy_s,
             "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99)),
             "queue_wait_ms_p50": float(np.percentile(wait, 50)), "queue_wait_ms_p99": float(np.percentile(wait, 99)),
             "failed": int(stats["failed"])}
        runs.append(r)
        log(f"  [served load {label}] offered {r['offered_rate_per_s']:.2f} req/s: {steps} steps in "
            f"{wall:.1f} s (busy {busy_s:.1f} s), capacity {r['steps_per_s_capacity']:.0f} steps/s "
            f"{r['requests_per_s_capacity']:.2f} req/s, p50 {r['latency_ms_p50']:.0f} ms "
            f"p99 {r['latency_ms_p99']:.0f} ms")
    out["runs"] = runs
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="ac3d_n1024")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison legs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the batched and served samples")
    ap.add_argument("--no-ps", action="store_true", help="skip the (p, s) sweep")
    ap.add_argument("--no-actd", action="store_true", help="skip the full-solve fallback leg")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the 2D 128^2 and 3D 256^3 workload legs")
    ap.add_argument("--init", choices=["warm", "hash"], default="warm",
                    help="initial guess of a mode: mode m of u^k (warm) or the counter-based vector")
    ap.add_argument("--no-alt-init", action="store_true", help="skip the leg with the other initial guess")
    ap.add_argument("--only", choices=["actd", "batched", "served", "ps", "ac2d", "ac3d_n256",
                                       "served_load", "mxy_alternatives"],
                    help="run only this leg and print its JSON (profiling aid; not the benchmark line)")
    ap.add_argument("--requests", type=int, default=64,
                    help="requests of the served workload for --only served_load")
    ap.add_argument("--batch-steps", type=int, default=2,
                    help="steps of every instance in --only batched")
    ap.add_argument("--batch-executors", default="lockstep,streams",
                    help="executors of the batched leg run by --only batched (comma-separated)")
    ap.add_argument("--no-lockstep", action="store_true",
                    help="served workload: every request on the worker-stream route")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="MIB",
                    help="first run the plain copy kernel on MIB MiB (scale for traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the CTD step of one instance is not sharded "
              "across GPUs; independent instances would run one server per GPU.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    from paper_2410_15519_amd import ctd
    from workloads import make_instance

    if args.copy_calibration > 0:
        nb = int(args.copy_calibration * 2 ** 20) // 16 * 16
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        ctd.kernel_copy(dst, src)
        torch.cuda.synchronize()
        assert torch.equal(dst, src)
        del src, dst
        torch.cuda.empty_cache()
    if args.only:
        legs = {"actd": lambda c: actd_leg(c),
                "batched": lambda c: batched_leg(c, init=args.init, steps=args.batch_steps,
                                                 executors=tuple(args.batch_executors.split(","))),
                "served": lambda c: served_leg(c, init=args.init),
                "ps": lambda c: ps_sweep_leg(c, init=args.init),
                "ac2d": lambda c: ac2d_leg(c), "ac3d_n256": lambda c: ac3d_n256_leg(c),
                "mxy_alternatives": lambda c: mxy_alternatives_leg(c),
                "served_load": lambda c: served_load_leg(c, count=args.requests, init=args.init,
                                                          lockstep=not args.no_lockstep)}
        print(json.dumps({args.only: legs[args.only](ctd)}))
        return
    inst = make_instance(args.workload)
    log(f"workload {args.workload}: dim={inst.dim} nodes={inst.nodes} eps={inst.eps} dt={inst.dt} "
        f"max_modes={inst.max_modes}")

    # leg 1: mixed, adaptive (the headline)
    warm_infos = []
    s_mix, infos, elapsed, prof, dec_all = run_leg(ctd, inst, "mixed", args.warmup, args.steps,
                                                   init=args.init, warm_infos=warm_infos)
    step0 = (warm_infos[0]["ms"], warm_infos[0]["sweeps"]) if warm_infos else (None, None)
    value = args.steps / elapsed
    dom, roof = roofline_of(prof["timed"], "mixed", args.workload)
    sweeps_per_step = float(np.mean([i["sweeps"] for i in infos]))
    extra = {"kernels_last_warmup_step": {
                 k: {"launches": v["launches"], "ms_total": round(v["ms"], 3),
                     "avg_us": round(1e3 * v["ms"] / v["launches"], 2)}
                 for k, v in prof["warmup"].items()},
             "modes_per_step": float(np.mean([i["modes"] for i in infos])),
             "sweeps_per_step": sweeps_per_step,
             "energy_last": infos[-1]["energy"]}
    fp64 = None
    if not args.no_fp64:
        n = int(np.prod(inst.nodes))
        Umix = torch.empty(n, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s_mix.reconstruct("f64", out=Umix)
        torch.cuda.synchronize()
        rec_s = time.perf_counter() - t0
        nm = int(s_mix.modes()[0].size)
        extra["reconstruct_f64"] = {"ms": rec_s * 1e3, "nodes": n, "modes": nm,
                                    "GB_per_s_written": 8.0 * n / rec_s / 1e9,
                                    "TFLOP_per_s": 2.0 * n * nm / rec_s / 1e12}
        log(f"  reconstruction of the 1024^3 field (f64, on device): {rec_s * 1e3:.1f} ms")
        # the FP32 field (FP32 MFMA): timed, then checked against the FP64 one
        U32 = torch.empty(n, dtype=torch.float32, device="cuda")
        s_mix.reconstruct("f32", out=U32)   # first call: kernel set-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s_mix.reconstruct("f32", out=U32)
        torch.cuda.synchronize()
        rec32 = time.perf_counter() - t0
        err32 = float(torch.linalg.norm(U32.double() - Umix) / torch.linalg.norm(Umix))
        extra["reconstruct_f32"] = {"ms": rec32 * 1e3, "nodes": n, "modes": nm,
                                    "GB_per_s_written": 4.0 * n / rec32 / 1e9,
                                    "TFLOP_per_s": 2.0 * n * nm / rec32 / 1e12,
                                    "rel_l2_vs_f64": err32}
        log(f"  reconstruction (f32, FP32 MFMA): {rec32 * 1e3:.1f} ms, rel l2 vs f64 {err32:.2e}")
        del U32
        torch.cuda.empty_cache()
        s_mix.close()
        del s_mix
        # leg 2: FP64 adaptive (timed for context); keep u^k before its last step
        s64 = ctd.Solver(inst, precision="fp64", energy=True, init=args.init)
        for k in range(args.warmup + args.steps - 1):
            s64.step(1)
        amp_prev, fac_prev = s64.modes()
        k_prev = s64.step_index
        s64.close()
        s64, infos64, el64, prof64, dec64 = run_leg(ctd, inst, "fp64", args.warmup, args.steps,
                                                    init=args.init)
        fp64 = {"steps_per_s": args.steps / el64,
                "dominant": roofline_of(prof64["timed"], "fp64", args.workload)[1]}
        U64 = torch.empty(n, dtype=torch.float64, device="cuda")
        s64.reconstruct("f64", out=U64)
        s64.close()
        # leg 3a: one mixed step from the FP64 state u^k with the FP64 step's decisions
        from workloads import Instance
        st = Instance(dim=inst.dim, nodes=inst.nodes, eps=inst.eps, S=inst.S, dt=inst.dt,
                      steps=1, amp=amp_prev, factors=fac_prev, max_modes=inst.max_modes,
                      seed=inst.seed, enrich_tol=inst.enrich_tol)
        one = ctd.Solver(st, precision="mixed", schedule="replay", init=args.init)
        one.step_index = k_prev
        one.set_decisions(dec64[-1:])
        one.step(1)
        U1 = torch.empty(n, dtype=torch.float64, device="cuda")
        one.reconstruct("f64", out=U1)
        one.close()
        fp64["rel_l2_step_mixed_vs_fp64"] = float(torch.linalg.norm(U1 - U64) / torch.linalg.norm(U64))
        del U1
        # leg 3d: the same single step in FP64 from u^k with amplitudes perturbed by 1e-14
        stp = Instance(**{**st.__dict__, "amp": amp_prev * (1.0 + 1e-14)})
        onep = ctd.Solver(stp, precision="fp64", schedule="replay", init=args.init)
        onep.step_index = k_prev
        onep.set_decisions(dec64[-1:])
        onep.step(1)
        U1 = torch.empty(n, dtype=torch.float64, device="cuda")
        onep.reconstruct("f64", out=U1)
        onep.close()
        fp64["rel_l2_step_fp64_uk_perturbed_1e-14"] = float(torch.linalg.norm(U1 - U64) / torch.linalg.norm(U64))
        del U1
        # leg 3b: accumulated difference of the mixed run against FP64 replaying its decisions
        sref, _, _, _, _ = run_leg(ctd, inst, "fp64", 0, args.warmup + args.steps,
                                   decisions=dec_all, profile=False, init=args.init)
        Uref = torch.empty(n, dtype=torch.float64, device="cuda")
        sref.reconstruct("f64", out=Uref)
        sref.close()
        fp64["rel_l2_accum_mixed_vs_fp64"] = float(torch.linalg.norm(Umix - Uref) / torch.linalg.norm(Uref))
        del Umix
        # leg 3c: intrinsic divergence of the truncated decomposition: FP64 replay
        # of the same decisions from u0 with amplitudes perturbed by 1e-14
        pert = Instance(**{**inst.__dict__, "amp": inst.amp * (1.0 + 1e-14)})
        sp, _, _, _, _ = run_leg(ctd, pert, "fp64", 0, args.warmup + args.steps,
                                 decisions=dec_all, profile=False, init=args.init)
        Up = torch.empty(n, dtype=torch.float64, device="cuda")
        sp.reconstruct("f64", out=Up)
        sp.close()
        fp64["rel_l2_accum_fp64_u0_perturbed_1e-14"] = float(torch.linalg.norm(Up - Uref) / torch.linalg.norm(Uref))
        fp64["accuracy_steps"] = args.warmup + args.steps
        del Up, Uref, U64
        torch.cuda.empty_cache()
        # leg 3e: the arithmetic of the mixed cubic contraction alone, at the
        # benchmarked size and mode count: the projected load of each
        # direction for 128 seeded modes and a seeded factor, mixed against FP64
        inst128 = make_instance(args.workload, m0=inst.max_modes)
        rng = np.random.default_rng(17)
        uu = [rng.uniform(-1.0, 1.0, int(m)) for m in inst128.nodes]
        loads = {}
        for prec in ("mixed", "fp64"):
            with ctd.Solver(inst128, precision=prec) as sl:
                loads[prec] = [sl.nonlinear_load(d, uu) for d in range(inst128.dim)]
        fp64["rel_l2_cubic_load_mixed_vs_fp64"] = max(
            float(np.linalg.norm(a - b) / np.linalg.norm(b)) for a, b in zip(loads["mixed"], loads["fp64"]))
        fp64["cubic_load_modes"] = int(inst.max_modes)
        del loads, inst128
    batched = served = None
    if not args.no_serve:
        batched = batched_leg(ctd, init=args.init)
        served = served_leg(ctd, init=args.init)
    ps_sweep = None if args.no_ps else ps_sweep_leg(ctd, init=args.init)
    other = "hash" if args.init == "warm" else "warm"
    alt_init = None if args.no_alt_init else init_leg(ctd, inst, args.warmup, args.steps, other)
    actd = None if args.no_actd else actd_leg(ctd)
    workloads = None
    if not args.no_workloads:
        workloads = {"ac2d_n128": ac2d_leg(ctd), "ac3d_n256": ac3d_n256_leg(ctd),
                     "mxy_alternatives_2d_n1024": mxy_alternatives_leg(ctd)}
    cpu = None if args.no_cpu_baseline else cpu_baseline(inst, step0[0], step0[1])
    out = {
        "metric": "CTD steps/s at 3D 1024^3 (mixed vs FP64, rel L2<=1e-6); served p50/p99 latency",
        "value": value, "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 / value, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp32-mfma+fp64",
        "data": "synthetic",
        "config": {"workload": args.workload, "dim": inst.dim, "nodes": list(inst.nodes),
                   "eps": inst.eps, "S": inst.S, "dt": inst.dt, "max_modes": inst.max_modes,
                   "precision": "mixed", "init_modes": int(len(inst.amp)), "s": inst.patch_s,
                   "p": inst.poly_p, "a": inst.dilation_a, "init": args.init},
        "roofline": roof,
        "cpu_baseline": cpu,
        "fp64": fp64,
        "served": served,
        "batched": batched,
        "ps_sweep": ps_sweep,
        "alt_init": alt_init,
        "actd": actd,
        "workloads": workloads,
        "detail": extra,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
