#!/usr/bin/env python
"""Benchmark of the batched multi-Debye fitting hot path on one MI355X.

One step = one whole fit of the mixed-material workload (1024 materials of
the HN / Cole-Cole / Cole-Davidson / Jonscher / CRIM families, F = 1000
log-spaced points on 1e6-1e10 Hz, N = 8 poles, 256 particles x 200 swarm
iterations), all on the GPU with inputs resident in HBM:
  target synthesis -> swarm init -> 201 batched cost evaluations interleaved
  with 200 swarm moves -> final bests -> L-BFGS polish of each material's
  best (adjoint gradients, batched Armijo trials).
value = cost evaluations per second over the step (forward evaluations of the
swarm and of the line-search trials, plus forward+adjoint evaluations of the
polish).  The JSON line also carries the kernel-only forward and
forward+adjoint rates, the roofline of the dominant kernel (the N = 8 cost
kernel, timed with HIP events on its stream), a parity check of a sampled
batch against the oracle, and the oracle's own rate on the host cores.

Usage: python bench.py [--gpus 1] [--steps 3] [--warmup 1]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VALU = 78.6e12   # 256 CUs x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
PEAK_HBM = 8.0e12


def algorithmic_flops(F, N):
    """Useful FP64 work of one cost evaluation, basis counted once:
    basis 5FN, Gram FN(N+1), rhs 2FN, column sums FN, residuals 4FN + F,
    cost 4F, dense solve N^3/3 + 2N^2."""
    return F * (N * N + 13 * N + 5) + N ** 3 / 3 + 2 * N * N


def algorithmic_bytes(F, N, P_per_mat):
    """HBM bytes one evaluation must move: its log10(tau) row in, cost out,
    and its share of the material's three spectra."""
    return 8 * N + 8 + 24 * F / P_per_mat


def kernel_source_hash():
    import hashlib
    # the cost kernel's own source: its file and the device helpers it includes
    src = b"".join(open(os.path.join(ROOT, "paper_2109_01928_amd", "csrc", f), "rb").read()
                   for f in ("fit_kernel.hpp", "fit_eval.hip", "common.hpp"))
    return hashlib.sha256(src).hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mixed", choices=["mixed", "single", "ragged", "hncc", "tables"],
                    help="mixed (default): 1024 mixed materials, F=1000, N=8, 256x200; single: one HN, F=50, N=5, "
                         "40x50; ragged: 4096 materials of uneven F/N/swarm size; hncc: 1024 HN/CC, F=2000, N=12; "
                         "tables: 65536 HN-sum tables, F=4096, N=20, 128 particles")
    ap.add_argument("--optimizer", default="pso", choices=["pso", "de", "da"],
                    help="global search: particle swarm (default), differential evolution (rand/1/bin) or "
                         "annealing (batched generalized simulated annealing chains)")
    ap.add_argument("--materials", type=int, default=0, help="override the workload's material count")
    ap.add_argument("--iters", type=int, default=-1, help="override the workload's swarm iterations")
    ap.add_argument("--polish-steps", type=int, default=-1)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--per-material", type=int, default=0,
                    help="also time the plain per-material loop (one material per launch sequence, forward only, "
                         "same swarm) on this many materials until each reaches the batched run's final cost, "
                         "capped at 10x the iterations, extrapolated to all materials")
    ap.add_argument("--no-autotune", action="store_true", help="keep the plan's default frequency splits")
    ap.add_argument("--freq-split", type=int, default=0,
                    help="fixed frequency split for every pole count (implies --no-autotune)")
    ap.add_argument("--only-eval", type=int, default=0,
                    help="profiling: run this many forward launches of the swarm batch and exit")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="profiling: time a device-to-device copy of this many bytes (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the fit shards by material with no communication, "
              "so the per-GPU rate is the figure; run it with --gpus 1 on a single MI355X.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2109_01928_amd as D
    import workloads as W

    dev = "cuda:0"
    torch.cuda.set_device(0)
    if args.copy_bytes:
        src = torch.ones(args.copy_bytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 8, "launches": 5}), flush=True)
        return
    wl = make_workload(W, args)
    args.iters = wl.iters
    if args.polish_steps < 0:
        args.polish_steps = wl.polish_steps
    M, P = wl.M, wl.P
    uniform = len(set(np.diff(wl.f_off))) == 1 and len(set(wl.n_poles)) == 1
    N = int(wl.n_poles.max())
    F = int(np.max(np.diff(wl.f_off)))
    P_per = int(np.max(np.diff(wl.cand_off)))
    T_TRIALS, MEM = 30, 10

    # static inputs resident in HBM before timing
    zeros = torch.zeros(len(wl.omega), dtype=torch.float64, device=dev)
    b = D.Batch(wl.f_off, wl.cand_off, wl.n_poles, wl.omega, zeros, zeros, dev)
    b1 = D.Batch(wl.f_off, np.arange(M + 1), wl.n_poles, b.omega, zeros, zeros, dev)
    kind_t = torch.tensor(wl.kind, dtype=torch.int8, device=dev)
    params_t = torch.tensor(wl.params, dtype=torch.float64, device=dev)
    lb = torch.tensor(wl.lb, device=dev)
    ub = torch.tensor(wl.ub, device=dev)
    plan = D.Plan(b)
    if args.freq_split:
        plan.set_freq_split(args.freq_split)
    elif not args.no_autotune:
        # schedule tuned once on the workload's own targets and a uniform draw of
        # candidates (set-up, outside the timed region)
        er0, ei0 = D.material_eval(kind_t, params_t, b, noise_seed=wl.noise_seed)
        th0 = torch.tensor(W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=5), device=dev)
        plan.autotune(b.with_targets(er0, ei0), th0, reps=2)
        del er0, ei0, th0
    sw = D.Swarm.empty(P, M, wl.ld, args.iters + 1, dev)
    work_per_eval = float(np.sum(np.diff(wl.cand_off) * np.array(
        [algorithmic_flops(int(f), int(n)) for f, n in zip(np.diff(wl.f_off), wl.n_poles)])))  # per swarm launch
    out = (torch.empty(P, dtype=torch.float64, device=dev), None, None, torch.empty(P, dtype=torch.int8, device=dev))
    stream = torch.cuda.current_stream()

    if args.only_eval:
        er, ei = D.material_eval(kind_t, params_t, b, noise_seed=wl.noise_seed)
        bb = b.with_targets(er, ei)
        theta = torch.tensor(W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=77), device=dev)
        for _ in range(args.only_eval):
            D.fit_eval(plan, bb, theta, want_weights=False, out=out)
        torch.cuda.synchronize()
        print(json.dumps({"launches": args.only_eval, "evals_per_launch": P, "flops_per_eval": algorithmic_flops(F, N),
                          "alg_bytes_per_eval": algorithmic_bytes(F, N, 256)}), flush=True)
        return

    pop = D.Population.empty(P, M, wl.ld, args.iters + 1, dev) if args.optimizer in ("de", "da") else None

    def timed_eval(bb, theta, evs, events):
        if events is not None:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
        D.fit_eval(plan, bb, theta, want_weights=False, out=out)
        if events is not None:
            e1.record(stream)
            evs.append((e0, e1))

    final = [None]   # each material's fitted log10 tau of the last step

    def one_step(events=None):
        er, ei = D.material_eval(kind_t, params_t, b, noise_seed=wl.noise_seed)
        bb = b.with_targets(er, ei)
        evs = []
        if args.optimizer == "de":
            D.de_init(bb, lb, ub, pop, seed=wl.seed)
            timed_eval(bb, pop.x, evs, events)
            D.de_select(bb, pop, 0, pop.x, out[0])
            for t in range(1, args.iters + 1):
                D.de_trial(bb, lb, ub, pop, t, seed=wl.seed)
                timed_eval(bb, pop.u, evs, events)
                D.de_select(bb, pop, t, pop.u, out[0])
            best = pop.best_x
        elif args.optimizer == "da":
            D.da_init(bb, lb, ub, pop, seed=wl.seed)
            timed_eval(bb, pop.x, evs, events)
            D.da_accept(bb, pop, 0, pop.x, out[0], seed=wl.seed)
            for t in range(1, args.iters + 1):
                D.da_visit(bb, lb, ub, pop, t, seed=wl.seed)
                timed_eval(bb, pop.u, evs, events)
                D.da_accept(bb, pop, t, pop.u, out[0], seed=wl.seed)
            best = pop.best_x
        else:
            D.pso_init(bb, lb, ub, sw, wl.inertia, wl.c1, wl.c2, wl.seed)
            for t in range(args.iters + 1):
                if t > 0:
                    D.pso_step(bb, lb, ub, sw, t, True, out[0], wl.inertia, wl.c1, wl.c2, wl.seed)
                timed_eval(bb, sw.x, evs, events)
            D.pso_step(bb, lb, ub, sw, args.iters + 1, False, out[0], wl.inertia, wl.c1, wl.c2, wl.seed)
            best = sw.gbest_x
        hist = None
        final[0] = best.clone()
        if args.polish_steps > 0:
            hist = D.lbfgs_polish(b1.with_targets(er, ei), final[0], lb, ub, steps=args.polish_steps, mem=MEM,
                                  max_trials=T_TRIALS)
        if events is not None:
            events.extend(evs)
        return er, ei, hist

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    events = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        er, ei, hist = one_step(events)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = 1e3 * dt / args.steps

    evals_swarm = P * (args.iters + 1)
    evals_polish = M * args.polish_steps * T_TRIALS + M * (args.polish_steps + 1) if args.polish_steps else 0
    evals_step = evals_swarm + evals_polish
    value = evals_step * args.steps / dt

    # dominant kernel: the swarm's cost evaluation, timed on its stream
    durs = np.array([a.elapsed_time(c) for a, c in events]) * 1e-3
    avg = float(durs.mean())
    wb = work_per_eval / P
    achieved = work_per_eval / avg
    fwd_rate = P / avg

    # the same swarm fit replayed from a captured HIP graph vs eager launches
    bbx = b.with_targets(er, ei)
    t_sw = {}
    def whole_fit(mode):
        if args.optimizer == "de":
            D.de_run(plan, bbx, lb, ub, pop, args.iters, seed=wl.seed, use_graph=mode)
        elif args.optimizer == "da":
            D.da_run(plan, bbx, lb, ub, pop, args.iters, seed=wl.seed, use_graph=mode)
        else:
            D.pso_run(plan, bbx, lb, ub, sw, args.iters, wl.inertia, wl.c1, wl.c2, wl.seed, use_graph=mode)

    for mode in (False, True):
        whole_fit(mode)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        whole_fit(mode)
        torch.cuda.synchronize()
        t_sw["graph" if mode else "eager"] = 1e3 * (time.perf_counter() - t1)

    # forward + adjoint kernel rate on the final swarm positions
    bb = b.with_targets(er, ei)
    theta = (pop.x if pop is not None else sw.x).clone()
    D.fit_eval_grad(plan, bb, theta)
    torch.cuda.synchronize()
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    g0.record(stream)
    for _ in range(reps):
        D.fit_eval_grad(plan, bb, theta)
    g1.record(stream)
    torch.cuda.synchronize()
    adj_rate = P * reps / (g0.elapsed_time(g1) * 1e-3)

    # HBM bytes per launch measured by rocprofv3 counters (profiles/); used only
    # while the kernel source is the one the counters were taken on
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "fit_eval_N8_mixed_traffic.json")
    if args.workload == "mixed" and os.path.exists(tfile):
        rec = json.load(open(tfile))
        split = str(plan.info()[0]["freq_split"])
        if rec.get("source_sha256_16") == kernel_source_hash() and split in rec.get("by_freq_split", {}):
            traffic = rec["by_freq_split"][split]["bytes"]

    line = {
        "metric": "Debye-fit cost evals/s (fwd, fwd+adjoint), rel err <=1e-10 vs FP64 oracle",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded materials; no dataset in the paper)",
        "config": {"workload": f"{wl.name} {args.optimizer.upper()} + L-BFGS polish {args.polish_steps} steps x "
                               f"{T_TRIALS} trials",
                   "materials": M, "freq_points": F if uniform else "ragged", "poles": N if uniform else "ragged",
                   "particles": P_per if uniform else "ragged", "iterations": args.iters,
                   "evals_per_step": evals_step},
        "fwd_kernel_evals_per_s": fwd_rate,
        "fwd_adjoint_kernel_evals_per_s": adj_rate,
        "swarm_fit_ms": {"eager": t_sw["eager"], "graph": t_sw["graph"]},
        "schedule": {f"N{i['n_poles']}": f"{i['pole_split']}x{i['freq_split']} lanes" for i in plan.info()},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU, "traffic": traffic,
                     "kernel": (f"fit_kernel<{N},{plan.info()[0]['pole_split']},false,"
                                f"{(1 if plan.info()[0]['freq_split'] == 1 else 2) if plan.info()[0]['uniform'] else 0}>")
                     if uniform else "fit_kernel (all pole-count buckets of one evaluation)",
                     "avg_launch_s": avg, "flops_per_eval": wb, "evals_per_launch": P},
    }
    # fit quality of the last step: average fractional error (Sec. IV) of each material's result
    b1t = b1.with_targets(er, ei)
    c1, w1, e1, _ = D.fit_eval(D.Plan(b1t), b1t, final[0])
    afe = D.afe(b1t, final[0], w1, e1).cpu().numpy()
    line["fit_quality"] = {"afe_percent_median": float(np.median(afe)), "afe_percent_max": float(np.max(afe)),
                           "afe_below_5_percent": float(np.mean(afe < 5.0))}
    if hist is not None:
        h = hist.cpu().numpy()
        drop = 1 - h[:, -1] / h[:, 0]
        line["polish"] = {"median_rel_cost_drop": float(np.median(drop)), "min_rel_cost_drop": float(drop.min()),
                          "monotone": bool(np.all(np.diff(h, axis=1) <= 0))}

    if args.per_material:
        line["per_material_loop"] = per_material_loop(D, wl, er, ei, c1.cpu().numpy(), args, ms_per_step / 1e3)

    if not args.no_cpu_baseline:
        line["cpu_baseline"], line["parity_sample"] = cpu_leg(D, W, wl, bb, plan, args.cpu_seconds)
        # counted evaluations: only those within the parity tolerance (sampled rate)
        ps = line["parity_sample"]
        line["value_raw"] = value
        line["value"] = value * ps["within_1e-10"] / ps["candidates"]
    print(json.dumps(line), flush=True)


def per_material_loop(D, wl, er, ei, target, args, batched_s):
    """The plain per-material alternative to the batched fit: each material
    alone (its own plan and swarm, forward evaluations only, the host reading
    the best cost after every iteration) iterates until its best cost is within
    1e-3 of the batched run's final (polished) cost, or 10x the iterations."""
    import torch

    cap = 10 * wl.iters
    times, reached, iters_used = [], 0, []
    for m in range(min(args.per_material, wl.M)):
        f0, f1 = int(wl.f_off[m]), int(wl.f_off[m + 1])
        P, N = int(wl.cand_off[m + 1] - wl.cand_off[m]), int(wl.n_poles[m])
        bm = D.Batch([0, f1 - f0], [0, P], [N], wl.omega[f0:f1], er[f0:f1].contiguous(), ei[f0:f1].contiguous())
        plan = D.Plan(bm)
        sw = D.Swarm.empty(P, 1, N, cap + 2)
        lbm = torch.tensor(wl.lb[m:m + 1], device="cuda")
        ubm = torch.tensor(wl.ub[m:m + 1], device="cuda")
        goal = target[m] * (1 + 1e-3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        D.pso_init(bm, lbm, ubm, sw, wl.inertia, wl.c1, wl.c2, wl.seed)
        cost = D.fit_eval(plan, bm, sw.x, want_weights=False)[0]
        t, best = 0, float("inf")
        while best > goal and t < cap:
            t += 1
            D.pso_step(bm, lbm, ubm, sw, t, True, cost, wl.inertia, wl.c1, wl.c2, wl.seed)
            cost = D.fit_eval(plan, bm, sw.x, want_weights=False)[0]
            best = float(sw.gbest_cost.item())
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        reached += best <= goal
        iters_used.append(t)
    k = len(times)
    est = float(np.mean(times)) * wl.M
    return {"materials_timed": k, "extrapolated_s": est, "batched_step_s": batched_s,
            "batched_speedup": est / batched_s, "reached_batched_cost": f"{reached}/{k}",
            "median_iterations": float(np.median(iters_used)), "iteration_cap": cap,
            "note": "extrapolated linearly from the timed materials; forward only (no adjoint polish)"}


def make_workload(W, args):
    if args.workload == "mixed":
        wl = W.mixed_uniform(M=args.materials or 1024, iters=args.iters if args.iters >= 0 else 200)
    elif args.workload == "single":
        wl = W.single_hn()
    elif args.workload == "ragged":
        wl = W.mixed_ragged(M=args.materials or 4096, iters=args.iters if args.iters >= 0 else 300)
    elif args.workload == "hncc":
        wl = W.hn_cc(M=args.materials or 1024, iters=args.iters if args.iters >= 0 else 200)
    else:
        wl = W.tables(M=args.materials or 65536, iters=args.iters if args.iters >= 0 else 400)
    if args.iters >= 0:
        wl.iters = args.iters
    return wl


def cpu_leg(D, W, wl, bb, plan, seconds):
    """Oracle on the host cores (bounded sample of whole materials, in order,
    until `seconds` of oracle time) and a parity check of the same sample on
    the GPU with the oracle's judgement: cost within 1e-10 of the FP64 oracle,
    or of its 80-bit instance, or within the cost's FP64 rounding sensitivity
    (oracle.judge_costs)."""
    import torch

    import oracle

    er = bb.eps_re.cpu().numpy()
    ei = bb.eps_im.cpu().numpy()
    # GPU targets vs oracle targets (target synthesis), then identical targets for the cost
    oer, oei = oracle.material_eval(wl.kind, wl.params, wl.f_off, wl.omega, noise_seed=wl.noise_seed)
    tgt_err = float(max(np.max(np.abs(er - oer) / np.maximum(np.abs(oer), 1e-300)),
                        np.max(np.abs(ei - oei) / np.maximum(np.abs(oei), 1e-300))))
    theta = W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=77)
    nthreads = oracle.num_threads()

    def sub_batch(m0, m1):
        f0, f1 = wl.f_off[m0], wl.f_off[m1]
        return oracle.Batch(wl.f_off[m0:m1 + 1] - f0, wl.cand_off[m0:m1 + 1] - wl.cand_off[m0], wl.n_poles[m0:m1],
                            wl.omega[f0:f1], oer[f0:f1], oei[f0:f1])

    # timed sample: whole materials in order; after the last material the
    # candidates are drawn again with the next seed, until `seconds`
    done_m, t_cpu, costs, n_timed, draw = 0, 0.0, [], 0, 0
    while t_cpu < seconds:
        m1 = min(done_m + 16, wl.M)
        th_all = theta if draw == 0 else W.draw_theta(wl.cand_off, wl.n_poles, wl.lb, wl.ub, wl.ld, seed=77 + draw)
        th = th_all[wl.cand_off[done_m]:wl.cand_off[m1]]
        t = time.perf_counter()
        c = oracle.fit_eval(sub_batch(done_m, m1), th, nthreads=nthreads)[0]
        t_cpu += time.perf_counter() - t
        n_timed += len(c)
        if draw == 0:
            costs.append(c)
        done_m = m1
        if done_m == wl.M:
            done_m, draw = 0, draw + 1
    n_draws = draw + (1 if done_m else 0)
    # the same oracle on one core, whole materials from the start, about a
    # fifth of the time budget
    m, t1, n1 = 0, 0.0, 0
    while t1 < seconds / 5 and m < wl.M:
        m1 = min(m + 2, wl.M)
        t = time.perf_counter()
        n1 += len(oracle.fit_eval(sub_batch(m, m1), theta[wl.cand_off[m]:wl.cand_off[m1]], nthreads=1)[0])
        t1 += time.perf_counter() - t
        m = m1
    c64 = np.concatenate(costs)
    n = len(c64)
    done_m = int(np.searchsorted(wl.cand_off, n))
    gb = bb.with_targets(torch.tensor(oer, device="cuda"), torch.tensor(oei, device="cuda"))
    cg = D.fit_eval(plan, gb, torch.tensor(theta, device="cuda"), want_weights=False)[0].cpu().numpy()[:n]
    per_m = np.array([np.sum(oer[wl.f_off[m]:wl.f_off[m + 1]] ** 2 + oei[wl.f_off[m]:wl.f_off[m + 1]] ** 2)
                      for m in range(done_m)])
    floor = 1e-12 * np.repeat(per_m, np.diff(wl.cand_off[:done_m + 1]))
    rel, judged = oracle.judge_costs(sub_batch(0, done_m), theta[:n], cg, c64, floor, 1e-10)
    cpu = {"value": n_timed / t_cpu, "unit": "evals/s", "cores": nthreads, "kind": "oracle",
           "sample": f"{n_timed} candidate evaluations of the same workload (whole materials in order, "
                     f"uniform log10 tau, {n_draws} draw(s)), Householder-QR FP64 oracle, "
                     f"{t_cpu:.1f} s; one core: {n1} evaluations in {t1:.1f} s",
           "value_1core": n1 / t1}
    parity = {"candidates": n, "max_cost_rel_err": float(rel.max()), "oracle_limited": judged["oracle_limited"],
              "fp64_limited": judged["fp64_limited"], "within_1e-10": int((rel <= 1e-10).sum()),
              "target_max_rel_err": tgt_err}
    return cpu, parity


if __name__ == "__main__":
    main()
