"""Throughput of full-batch SPFOM iterations on one MI355X.

A step is one whole SPFOM iteration (every row of the hot path: price step,
per-segment exact best response, fixed-point sales scatter, FP64
reductions, projected dual step) over the L=2e6-segment, n=2e4-product
Zipf workload with FP32 iterates and FP64 reductions.  Inputs are resident
in HBM before timing starts.

Prints one JSON line (stdout).  Progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BF16_PEAK = 2.5e15            # dense BF16 matrix-core peak of MI355X, FLOP/s
HBM_PEAK = 8.0e12          # MI355X HBM3E, bytes/s


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(inst, esz):
    """Bytes one segment-kernel launch must move: the CSR entries (product id
    4 B, v and w esz each), per segment the row pointer (8 B), vt0 and lambda
    (esz each), per product the price read (esz) and the sales
    accumulator (8 B).  Left out on purpose: what the library's own layout
    adds (the warm-start R* per segment it reads and writes, the padding of
    its slot-major copy, reported separately as slot_entries) - those are
    this implementation's choices, not bytes the method must move."""
    nnz, L, n = inst.nnz, inst.L, inst.n
    per_nnz = 4 + 2 * esz
    per_seg = 8 + 2 * esz
    per_prod = esz + 8
    return nnz * per_nnz + L * per_seg + n * per_prod, dict(per_nnz=per_nnz, per_seg=per_seg,
                                                            per_prod=per_prod)


PROFILE_OF = {"plain-L2e6-n2e4-zipf-identity": "k_segments-plain-L2e6-n2e4.md",
              "plain-L1e7-n1e5-m2e3-zipf-resources": "k_segments-plain-L1e7-n1e5-m2e3.md"}
# the segment kernel's sources; the profile records their hash
PROFILE_SOURCES = ("segment.hip", "segment_core.hpp", "common.hpp")


def profiled_traffic(workload):
    """HBM bytes per segment-kernel launch from the committed rocprofv3 summary
    (FETCH_SIZE and WRITE_SIZE, scaled by the copy calibration), or None when
    there is none for the workload or the kernel source changed since the
    counters were taken."""
    import hashlib
    name = PROFILE_OF.get(workload)
    path = os.path.join(ROOT, "profiles", name) if name else None
    if not path or not os.path.exists(path):
        return None
    src = b"".join(open(os.path.join(ROOT, "paper_2602_22421_amd", "csrc", f), "rb").read()
                   for f in PROFILE_SOURCES)
    sha = hashlib.sha256(src).hexdigest()[:16]
    rec, traffic = None, None
    for line in open(path):
        if line.startswith("source_sha256_16:"):
            rec = line.split()[1]
        if line.startswith("traffic_bytes_per_launch:"):
            traffic = float(line.split()[1])
    return traffic if rec == sha else None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _slice(inst, lo, hi):
    import dataclasses
    e0, e1 = int(inst.seg_ptr[lo]), int(inst.seg_ptr[hi])
    return dataclasses.replace(inst, L=hi - lo, seg_ptr=inst.seg_ptr[lo:hi + 1] - e0,
                               idx=inst.idx[e0:e1], v=inst.v[e0:e1], w=inst.w[e0:e1],
                               v0=inst.v0[lo:hi], lam=inst.lam[lo:hi])


def cpu_baseline(inst, tau, iters):
    """The FP64 oracle as it stands (single-threaded C) on the whole instance:
    `iters` iterations from eta = 0.  Returns the baseline record and the
    oracle's duals and trace (for the GPU's error at the same iteration)."""
    import oracle
    s = oracle.Solver(inst, tau=tau, check_every=10)
    t0 = time.perf_counter()
    eta, tr = s.iterate(np.zeros(inst.m), iters, trace=True)
    dt = time.perf_counter() - t0
    rec = {"value": inst.L * iters / dt, "unit": "segment-updates/s", "cores": 1,
           "kind": "oracle",
           "sample": f"{iters} FP64 iterations over all {inst.L} segments ({inst.nnz} CSR "
                     f"entries) of the same instance, single-threaded C, {dt:.1f} s",
           "cpu_model": cpu_model(), "nproc": os.cpu_count()}
    return rec, eta, tr


_POOL_INST = None


def _pool_leg(task):
    lo, hi, reps, tau = task
    import oracle
    sub = _slice(_POOL_INST, lo, hi)
    s = oracle.Solver(sub, tau=tau, check_every=10)
    t0 = time.perf_counter()
    s.iterate(np.zeros(sub.m), reps, trace=False)
    return hi - lo, reps, time.perf_counter() - t0


def cpu_baseline_all_cores(inst, tau, reps, workers):
    """The same oracle run by `workers` processes at once, each over its own
    contiguous share of the segments (the method's segments are independent
    within an iteration; each process also takes the cheap dual step on its
    share).  Throughput = all segments x reps / the slowest process's time."""
    import multiprocessing as mp
    global _POOL_INST
    _POOL_INST = inst
    cuts = [inst.L * k // workers for k in range(workers + 1)]
    tasks = [(cuts[k], cuts[k + 1], reps, tau) for k in range(workers)]
    with mp.get_context("fork").Pool(workers) as pool:
        out = pool.map(_pool_leg, tasks)
    _POOL_INST = None
    slowest = max(t for _, _, t in out)
    segs = sum(n for n, _, _ in out)
    return {"value": segs * reps / slowest, "unit": "segment-updates/s", "cores": workers,
            "kind": "oracle",
            "sample": f"{reps} FP64 iterations over all {inst.L} segments split into {workers} "
                      f"contiguous shares, one single-threaded oracle process per share, "
                      f"slowest share {slowest:.1f} s",
            "cpu_model": cpu_model(), "nproc": os.cpu_count()}


GAP_LEVELS = (1e-1, 3e-2, 1e-2, 3e-3, 1e-3, 3e-4, 1e-4)


def _run_to_levels(cblp, prob, eta, params, iters, chunk, t_start=0.0):
    """Iterate `iters` times from eta in chunks, recording the wall time of
    each chunk; returns (time and iterations to each certified gap level,
    final trace row, seconds per iteration).  The gap is read at the checks
    (every check_every iterations); a level's time is the chunk's start plus
    its share of the chunk up to that check."""
    import torch
    K = int(params.check_every)
    reach = {f"{lv:g}": None for lv in GAP_LEVELS}
    t = 0
    wall = t_start
    last = None
    while t < iters:
        n = min(chunk, iters - t)
        tr = np.zeros((n, cblp.NTRACE))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cblp.spfom_iterate(prob.h, eta, params, n, tr)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        for k in range(n):
            tt = t + k + 1
            if tt % K:
                continue
            for lv in GAP_LEVELS:
                key = f"{lv:g}"
                if reach[key] is None and tr[k, 7] <= lv:
                    reach[key] = {"iters": tt, "seconds": wall + dt * (k + 1) / n}
        wall += dt
        t += n
        last = tr[-1]
    return reach, last, (wall - t_start) / max(iters, 1)


def _schedule_params(cblp, prob, inst, args, tau0=None):
    from paper_2602_22421_amd.instances import step_scale
    npdt = np.float32 if prob.dtype.itemsize == 4 else np.float64
    tau = prob.tensor(step_scale(inst, args.tau0 if tau0 is None else tau0).astype(npdt))
    return cblp.make_params(rule=cblp.SPFOM_STEP_CONST, tau_vec=tau, check_every=10,
                            bound=cblp.SPFOM_BOUND_SEGMENT if args.bound == "segment"
                            else cblp.SPFOM_BOUND_GLOBAL,
                            tau_decay=args.tau_decay, decay_every=args.decay_every)


def time_to_gap(args):
    """Plain cold-start SPFOM on the L=2e6 workload: wall time and iterations
    to each certified relative gap level (the dual bound Dbest against the
    scaled averaged-primal bound), with the decaying constant step."""
    import torch
    from paper_2602_22421_amd import cblp
    from paper_2602_22421_amd.instances import CONFIG_NAMES, config_instance
    inst = config_instance(args.config).cast(np.float32)
    prob = cblp.Problem(inst, dtype=torch.float32)
    out_runs = []
    for bound in args.bounds:
        args.bound = bound
        params = _schedule_params(cblp, prob, inst, args)
        prob.reset()
        eta = prob.zeros_eta()
        reach, last, per = _run_to_levels(cblp, prob, eta, params, args.max_iters, 1000)
        log(f"bound {bound}: final gap {last[7]:.3e} after {args.max_iters} iterations, "
            f"{per * 1e3:.3f} ms/iteration; levels {reach}")
        out_runs.append({"bound": bound, "reach": reach, "final_gap": float(last[7]),
                         "dbest": float(last[5]), "lb": float(last[6]),
                         "ms_per_iter": per * 1e3})
    best = min(out_runs, key=lambda r: r["final_gap"])
    lv = f"{args.gap:g}"
    out = {
        "metric": f"time to certified gap {args.gap:g}, plain cold start", "unit": "s",
        "value": best["reach"][lv]["seconds"] if best["reach"].get(lv) else None,
        "higher_is_better": False, "n_gpus": 1, "dtype": "f32", "data": "synthetic",
        "vs_baseline": None,
        "config": {"workload": CONFIG_NAMES[args.config], "L": inst.L, "n": inst.n,
                   "nnz": inst.nnz, "step_rule": "const", "tau0": args.tau0,
                   "tau_decay": args.tau_decay, "decay_every": args.decay_every,
                   "check_every": 10, "max_iters": args.max_iters},
        "tightest_gap": best["final_gap"], "runs": out_runs,
    }
    print(json.dumps(out), flush=True)
    prob.close()


def batched(args):
    """Multi-period batch: for each certified gap level, the time for every
    instance to reach it (or the iteration cap), solved as one batch and one
    instance after another with spfom_solve; the same decaying constant step,
    checks and cap for both."""
    import torch
    from paper_2602_22421_amd import cblp
    from paper_2602_22421_amd.instances import batch_instance, step_scale

    t0 = time.perf_counter()
    insts = [batch_instance(b, scale=args.batch_scale).cast(np.float32)
             for b in range(args.batch_count)]
    nnz = sum(i.nnz for i in insts)
    L = sum(i.L for i in insts)
    log(f"generated {len(insts)} instances: sum L = {L}, sum nnz = {nnz} "
        f"in {time.perf_counter() - t0:.1f} s")
    levels = [float(x) for x in args.levels]

    def params_for(tol, tau_vec=None):
        return cblp.make_params(rule=cblp.SPFOM_STEP_CONST, tau=1.0, tau_vec=tau_vec,
                                check_every=10, tol=tol, max_iters=args.max_iters,
                                tau_decay=args.tau_decay, decay_every=args.decay_every)

    probs = [cblp.Problem(i, dtype=torch.float32) for i in insts]
    taus = [p.tensor(step_scale(i, args.tau0).astype(np.float32)) for p, i in zip(probs, insts)]
    batch = cblp.Batch(probs)
    variant = batch.tune([p.zeros_eta() for p in probs], params_for(levels[0]), iters=3,
                         tau_vecs=taus)
    runs = []
    for tol in levels:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        seq = []
        for p, t in zip(probs, taus):
            p.reset()
            seq.append(p.solve(p.zeros_eta(), params_for(tol, t)).as_dict())
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t0
        etas = [p.zeros_eta() for p in probs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs = batch.solve(etas, params_for(tol), tau_vecs=taus)
        torch.cuda.synchronize()
        t_bat = time.perf_counter() - t0
        run = {"tol": tol, "batched_s": t_bat, "sequential_s": t_seq, "speedup": t_seq / t_bat,
               "converged_batched": sum(o["status"] == 0 for o in outs),
               "converged_sequential": sum(o["status"] == 0 for o in seq),
               "iterations_batched": sum(o["iters"] for o in outs),
               "iterations_sequential": sum(o["iters"] for o in seq),
               "worst_gap_batched": max(o["gap"] for o in outs)}
        log(f"tol {tol:g}: batched {t_bat:.2f} s ({run['converged_batched']}/{len(outs)} "
            f"converged), sequential {t_seq:.2f} s ({run['converged_sequential']} converged)")
        runs.append(run)
    head = runs[-1]
    out = {
        "metric": f"time to certified gap {head['tol']:g}, all instances, batched",
        "value": head["batched_s"], "unit": "s",
        "higher_is_better": False, "n_gpus": 1, "dtype": "f32", "data": "synthetic",
        "vs_baseline": None,
        "config": {"workload": f"multi-period-batch-{len(insts)}", "instances": len(insts),
                   "sum_L": L, "sum_nnz": nnz, "max_iters": args.max_iters,
                   "check_every": 10, "step_rule": "const", "tau0": args.tau0,
                   "tau_decay": args.tau_decay, "decay_every": args.decay_every,
                   "batch_scale": args.batch_scale},
        "levels": runs, "tuned_variant": variant, "batch": batch.info(),
    }
    print(json.dumps(out), flush=True)
    batch.close()
    for p in probs:
        p.close()


def minibatch_bench(args):
    """Stochastic minibatch SPFOM on the L=2e6 workload: each iteration
    re-solves B sampled segments (an epoch walk through random permutations)
    and steps the duals with the kept sales of all segments.  Reports
    sampled-segment updates per second for each B."""
    import torch
    from paper_2602_22421_amd import cblp
    from paper_2602_22421_amd.instances import config_instance, minibatch_schedule, step_scale
    inst = config_instance(args.config).cast(np.float32)
    prob = cblp.Problem(inst, dtype=torch.float32)
    tau = prob.tensor(step_scale(inst, args.tau0).astype(np.float32))
    params = cblp.make_params(rule=cblp.SPFOM_STEP_CONST, tau_vec=tau, check_every=10)
    runs = []
    for frac in args.mb_fracs:
        B = max(1, int(round(inst.L * float(frac))))
        iters = args.steps
        sched = torch.from_numpy(minibatch_schedule(inst.L, B, args.warmup + iters, seed=7,
                                                    mode="epoch")).to(prob.device)
        prob.reset()
        eta = prob.zeros_eta()
        warm = sched[:args.warmup].contiguous()
        cblp.spfom_minibatch(prob.h, eta, params, warm, args.warmup)
        timed = sched[args.warmup:].contiguous()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cblp.spfom_minibatch(prob.h, eta, params, timed, iters)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / iters
        gap = prob.gap(eta)
        run = {"B": B, "fraction": float(frac), "ms_per_iter": dt * 1e3,
               "sampled_segment_updates_per_s": B / dt,
               "D_after": gap["D"], "iters": iters, "warmup": args.warmup}
        log(f"minibatch B={B}: {dt * 1e3:.3f} ms/iteration, {B / dt:.3e} segment-updates/s, "
            f"D {gap['D']:.6e}")
        runs.append(run)
    out = {"metric": "sampled segment-updates/s, stochastic minibatch SPFOM",
           "value": runs[0]["sampled_segment_updates_per_s"], "unit": "segment-updates/s",
           "higher_is_better": True, "n_gpus": 1, "dtype": "f32", "data": "synthetic",
           "vs_baseline": None,
           "config": {"workload": "plain-L2e6-n2e4-zipf-identity", "L": inst.L, "n": inst.n,
                      "nnz": inst.nnz, "sampler": "epoch permutations", "step_rule": "const",
                      "tau0": args.tau0},
           "runs": runs}
    print(json.dumps(out), flush=True)
    prob.close()


def recover_bench(args):
    """SBLP -> CBLP recovery on the L=2e6 workload: nested assortments and
    their probabilities from the per-entry sales of one best-response pass."""
    import torch
    from paper_2602_22421_amd import cblp
    from paper_2602_22421_amd.instances import config_instance, step_scale
    inst = config_instance(args.config).cast(np.float32)
    prob = cblp.Problem(inst, dtype=torch.float32)
    tau = prob.tensor(step_scale(inst, args.tau0).astype(np.float32))
    params = cblp.make_params(rule=cblp.SPFOM_STEP_CONST, tau_vec=tau, check_every=10)
    eta = prob.zeros_eta()
    prob.iterate(eta, 50, params)
    _, _, _, y = prob.sales(eta, entries=True)
    rank = torch.empty(inst.nnz, dtype=torch.int32, device=prob.device)
    alpha = torch.empty(inst.nnz, dtype=torch.float64, device=prob.device)
    alpha0 = torch.empty(inst.L, dtype=torch.float64, device=prob.device)
    for _ in range(3):
        cblp.cblp_recover(prob.h, y, rank, alpha, alpha0)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    reps = 20
    ev[0].record()
    for _ in range(reps):
        cblp.cblp_recover(prob.h, y, rank, alpha, alpha0)
    ev[1].record()
    torch.cuda.synchronize()
    us = ev[0].elapsed_time(ev[1]) * 1e3 / reps
    # bytes the recovery must move: y 8, v 4, w 4 in; rank 4, alpha 8 out per
    # entry; row pointer 8, v0 4, lambda 4 in, alpha0 8 out per segment
    nbytes = 28 * inst.nnz + 24 * inst.L
    log(f"recover: {us:.1f} us/call, {nbytes / us / 1e3:.0f} GB/s of {nbytes / 1e6:.1f} MB")
    out = {"metric": "SBLP to CBLP recovery time", "value": us, "unit": "us",
           "higher_is_better": False, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
           "vs_baseline": None,
           "config": {"workload": "plain-L2e6-n2e4-zipf-identity", "L": inst.L, "n": inst.n,
                      "nnz": inst.nnz, "sales": "best response after 50 iterations"},
           "roofline": {"bound": "hbm", "achieved": nbytes / us / 1e3, "peak": 8000.0,
                        "unit": "GB/s", "frac": nbytes / us / 1e3 / 8000.0,
                        "bytes_per_call": nbytes}}
    print(json.dumps(out), flush=True)
    prob.close()


def gosim_bench(args):
    """The GO bid-price policy on the market of Figure 4 (Section 5.1): runs
    independent runs of T batches of N customers over n products, K offered
    per batch; every batch with more than K products in stock re-solves its
    LP by SPFOM (all runs in one batched solve, warm-started from the
    previous batch's duals).  Reports simulated customers per second, the
    time per batch and the LP iterations; the oracle's closed loop, timed on
    a bounded sample, is the CPU baseline."""
    import torch
    from paper_2602_22421_amd import cblp
    from paper_2602_22421_amd.instances import gosim_market
    dt = torch.float32 if args.dtype == "f32" else torch.float64
    npdt = np.float32 if args.dtype == "f32" else np.float64
    t0 = time.perf_counter()
    mk = gosim_market(args.gs_runs, n=args.gs_products, periods=args.gs_periods,
                      customers=args.gs_customers, seed=0, dtype=npdt)
    log(f"market: {mk.runs} runs x {mk.periods} batches x {mk.customers} customers x "
        f"{mk.n} products in {time.perf_counter() - t0:.1f} s")
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import gosim as ogs
        kw = dict(tau0=args.gs_tau0, tol=args.gs_tol, max_iters=args.gs_max_iters,
                  check_every=10, rule=1 if args.gs_rule == "polyak" else 0,
                  tau_decay=args.gs_decay, decay_every=args.gs_decay_every)
        t0 = time.perf_counter()
        ogs.simulate(mk.r[0], mk.inv0[0], mk.prefs[:, 0], mk.u[:, 0], args.gs_k, batches=1, **kw)
        first = time.perf_counter() - t0
        done = int(max(1, min(mk.periods, args.oracle_seconds / max(first, 1e-3))))
        t0 = time.perf_counter()
        ogs.simulate(mk.r[0], mk.inv0[0], mk.prefs[:, 0], mk.u[:, 0], args.gs_k, batches=done,
                     **kw)
        el = time.perf_counter() - t0
        cpu = {"value": done * mk.customers / el, "unit": "customers/s", "cores": 1,
               "kind": "oracle",
               "sample": f"run 0 of the market, its first {done} of {mk.periods} batches "
                         f"({el:.1f} s, FP64)"}
        log(f"oracle: {cpu['value']:.3e} customers/s")
    sim = cblp.GoSim(mk, dtype=dt)
    cblp.cblp_batch_persistent(sim.b, args.gs_persistent)
    rule = cblp.SPFOM_STEP_POLYAK if args.gs_rule == "polyak" else cblp.SPFOM_STEP_CONST
    params = cblp.make_params(rule=rule, tau=1.0, check_every=10, tol=args.gs_tol,
                              max_iters=args.gs_max_iters, tau_decay=args.gs_decay,
                              decay_every=args.gs_decay_every)
    sim.run(args.gs_k, params, args.gs_tau0)          # warm-up: graph capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = sim.run(args.gs_k, params, args.gs_tau0)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    customers = mk.runs * mk.periods * mk.customers
    solved = out["lp_iters"] > 0
    cum = out["revenue"].sum(axis=0)
    # the same market without bid prices (duals held at zero: the K highest
    # prices in stock offered every batch), for scale
    zero = cblp.make_params(rule=cblp.SPFOM_STEP_CONST, tau=1.0, check_every=10, tol=0.0,
                            max_iters=0)
    flat = sim.run(args.gs_k, zero, args.gs_tau0)["revenue"].sum(axis=0)
    log(f"GO: {el:.2f} s for {mk.periods} batches x {mk.runs} runs ({customers / el:.3e} "
        f"customers/s); LPs solved in {solved.mean():.0%} of batches, "
        f"{out['lp_iters'][solved].mean() if solved.any() else 0:.0f} iterations each, median "
        f"gap {np.median(out['lp_gap'][solved]) if solved.any() else 0:.2e}; "
        f"revenue per run {cum.mean():.1f} (zero duals: {flat.mean():.1f})")
    res = {"metric": "simulated customers/s, GO bid-price policy with batched SPFOM re-solves",
           "value": customers / el, "unit": "customers/s", "higher_is_better": True,
           "n_gpus": 1, "dtype": args.dtype, "data": "synthetic", "vs_baseline": None,
           "ms_per_batch": el / mk.periods * 1e3,
           "config": {"workload": f"go-bid-price-{mk.runs}runs-{mk.periods}x{mk.customers}-"
                                  f"n{mk.n}-K{args.gs_k}",
                      "runs": mk.runs, "batches": mk.periods, "customers": mk.customers,
                      "products": mk.n, "K": args.gs_k, "tol": args.gs_tol,
                      "max_iters": args.gs_max_iters, "tau0": args.gs_tau0,
                      "step_rule": args.gs_rule, "tau_decay": args.gs_decay,
                      "decay_every": args.gs_decay_every, "persistent": args.gs_persistent},
           "lp": {"solved_fraction": float(solved.mean()),
                  "median_gap": float(np.median(out["lp_gap"][solved])) if solved.any() else 0.0,
                  "converged_fraction": float((out["lp_gap"][solved] <= args.gs_tol).mean())
                  if solved.any() else 0.0,
                  "mean_iters": float(out["lp_iters"][solved].mean()) if solved.any() else 0.0,
                  "max_iters_hit": int((out["lp_iters"] >= args.gs_max_iters).sum())},
           "revenue": {"mean_per_run": float(cum.mean()), "std_per_run": float(cum.std()),
                       "zero_duals_mean_per_run": float(flat.mean()),
                       "per_batch_mean": out["revenue"].mean(axis=1).round(3).tolist()},
           "cpu_baseline": cpu}
    print(json.dumps(res), flush=True)
    sim.close()


def _ws_train_instance(job):
    """One training instance of the learned warm start (run in a worker process)."""
    from paper_2602_22421_amd.instances import config_instance
    seed, L, caps = job
    return config_instance(1, seed=seed, L=L, cap_lo=caps[0], cap_hi=caps[1],
                           name=f"ws-train-{seed}").cast(np.float32)


def warmstart_bench(args):
    """Learned warm start on its stated workload: generate --ws-train
    instances of the L=2e6 Zipf generator at L=1e5 (n=2e4 products, the same
    capacity law), solve each from zero (decaying constant step, FP32
    iterate) and collect every product's features and dual; train the network
    on the GPU; then solve held-out L=2e6 instances from its prediction (the
    library's fallback to zero included) and from zero with the same step,
    recording the iterations and seconds each start needs to certify each gap
    level.  Instances are generated by worker processes (started fresh, not
    forked) while the GPU solves."""
    import multiprocessing as mp
    import torch
    from paper_2602_22421_amd import cblp, warmstart
    from paper_2602_22421_amd.instances import config_instance, step_scale

    caps = {"tight": (0.2, 0.5), "loose": (0.5, 3.0)}[args.ws_caps]
    train_L = 100_000
    t0 = time.perf_counter()
    jobs = [(10_000 + s, train_L, caps) for s in range(args.ws_train)]
    xs, ys, gaps = [], [], []
    workers = max(1, min(16, (os.cpu_count() or 2) - 1))
    with mp.get_context("spawn").Pool(workers) as pool:
        for k, inst in enumerate(pool.imap(_ws_train_instance, jobs)):
            prob = cblp.Problem(inst, dtype=torch.float32)
            tau = prob.tensor(step_scale(inst, args.ws_tau0).astype(np.float32))
            prm = cblp.make_params(rule=cblp.SPFOM_STEP_CONST, tau_vec=tau, check_every=10,
                                   tau_decay=args.tau_decay, decay_every=args.decay_every)
            eta = prob.zeros_eta()
            _, st = prob.iterate(eta, args.ws_target_iters, prm, trace=False)
            gaps.append(st.as_dict()["gap"])
            xs.append(cblp.features(prob))
            ys.append(cblp.targets(prob, eta))
            prob.close()
            if k % 64 == 0:
                log(f"collect {k}: gap {gaps[-1]:.3e} after {args.ws_target_iters} iterations "
                    f"({time.perf_counter() - t0:.1f} s)")
    X, Y = torch.cat(xs).contiguous(), torch.cat(ys).contiguous()
    del xs, ys
    t_collect = time.perf_counter() - t0
    log(f"collected {X.shape[0]} products from {args.ws_train} solved L=1e5, n=2e4 instances "
        f"in {t_collect:.1f} s (median target gap {np.median(gaps):.3e})")
    net = cblp.WarmStartNet(seed=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = warmstart.train(net, X, Y, epochs=args.ws_epochs, batch=16384, lr=3e-4)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"trained {args.ws_epochs} epochs in {t_train:.1f} s: loss {losses[0]:.3e} -> "
        f"{losses[-1]:.3e} (target variance {float(Y.var()):.3e})")
    # matrix-core throughput of the network: forward over every training row,
    # and one epoch of training steps (2 launches each)
    rows = X.shape[0]
    flops_fwd = 2.0 * rows * (4 * 256 + 256 * 256 + 256)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    net.forward(X)
    ev[0].record()
    for _ in range(5):
        net.forward(X)
    ev[1].record()
    ev[2].record()
    net.train(X, Y, epochs=1, batch=16384, lr=1e-6, seed=1)
    ev[3].record()
    torch.cuda.synchronize()
    fwd_s = ev[0].elapsed_time(ev[1]) / 5e3
    ep_s = ev[2].elapsed_time(ev[3]) / 1e3
    mlp = {"rows": rows, "forward_ms": fwd_s * 1e3,
           "forward_tflops": flops_fwd / fwd_s / 1e12,
           "forward_frac_bf16_peak": flops_fwd / fwd_s / BF16_PEAK,
           "train_epoch_ms": ep_s * 1e3, "train_batch": 16384,
           "train_tflops": 3.0 * flops_fwd / ep_s / 1e12,
           "train_frac_bf16_peak": 3.0 * flops_fwd / ep_s / BF16_PEAK}
    log(f"network: forward {fwd_s * 1e3:.2f} ms over {rows} rows "
        f"({mlp['forward_tflops']:.1f} TFLOP/s), training epoch {ep_s * 1e3:.1f} ms "
        f"({mlp['train_tflops']:.1f} TFLOP/s)")
    levels = (1e-1, 3e-2, 1e-2, 3e-3, 1e-3, 1e-4)
    results = []
    for seed in args.ws_eval_seeds:
        inst = config_instance(1, seed=seed, cap_lo=caps[0], cap_hi=caps[1]).cast(np.float32)
        prob = cblp.Problem(inst, dtype=torch.float32)
        tau = prob.tensor(step_scale(inst, args.ws_tau0).astype(np.float32))
        params = cblp.make_params(rule=cblp.SPFOM_STEP_CONST, tau_vec=tau, check_every=10,
                                  tau_decay=args.tau_decay, decay_every=args.decay_every)
        row = {"seed": seed}
        starts = ([f"cold-x{f:g}" for f in args.ws_cold_tau] +
                  [f"warm-x{f:g}" for f in args.ws_warm_tau])
        for start in starts:
            scale = float(start[6:])
            params = cblp.make_params(rule=cblp.SPFOM_STEP_CONST, tau_vec=tau * scale,
                                      check_every=10, tau_decay=args.tau_decay,
                                      decay_every=args.decay_every)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = {}
            if start.startswith("warm"):
                eta, info = net.start(prob)    # prediction and fallback, in the library
            else:
                eta = prob.zeros_eta()
            torch.cuda.synchronize()
            t_start = time.perf_counter() - t0
            prob.reset()
            tr = np.zeros((args.max_iters, cblp.NTRACE))
            t1 = time.perf_counter()
            cblp.spfom_iterate(prob.h, eta, params, args.max_iters, tr)
            torch.cuda.synchronize()
            per_iter = (time.perf_counter() - t1) / args.max_iters
            cgaps = tr[9::10, 7]
            reach = {}
            for lv in levels:
                k = np.nonzero(cgaps <= lv)[0]
                it = int((k[0] + 1) * 10) if len(k) else None
                reach[f"{lv:g}"] = None if it is None else {
                    "iters": it, "seconds": t_start + it * per_iter}
            row[start] = dict(info, reach=reach, final_gap=float(cgaps.min()),
                              dbest=float(tr[-1, 5]), start_seconds=t_start,
                              ms_per_iter=per_iter * 1e3)
            log(f"seed {seed} {start}: best gap {cgaps.min():.3e}, reach {reach}")
        results.append(row)
        prob.close()

    colds = [f"cold-x{f:g}" for f in args.ws_cold_tau]
    warms = [f"warm-x{f:g}" for f in args.ws_warm_tau]

    def mean_seconds(start, lv):
        v = [r[start]["reach"][lv] for r in results]
        return float(np.mean([x["seconds"] for x in v])) if all(v) else None

    def best_cold(lv):
        v = [x for x in (mean_seconds(c, lv) for c in colds) if x is not None]
        return min(v) if v else None

    def speedup(lv, warm):
        c, w = best_cold(lv), mean_seconds(warm, lv)
        return c / w if c and w else None

    reached = [f"{lv:g}" for lv in levels if best_cold(f"{lv:g}") and mean_seconds(warms[0], f"{lv:g}")]
    head = reached[-1] if reached else None
    out = {
        "metric": f"time to certified gap {head}, warm start ({warms[0]}) vs the fastest cold "
                  f"start of steps x{args.ws_cold_tau} (the tightest level both reach on every "
                  f"held-out instance)", "unit": "s",
        "value": mean_seconds(warms[0], head) if head else None,
        "cold_value": best_cold(head) if head else None,
        "levels_only_warm": [f"{lv:g}" for lv in levels
                             if mean_seconds(warms[0], f"{lv:g}") and not best_cold(f"{lv:g}")],
        "higher_is_better": False, "n_gpus": 1, "dtype": "f32", "data": "synthetic",
        "vs_baseline": None,
        "config": {"workload": f"warm-start-L2e6-n2e4-zipf-caps-{args.ws_caps}",
                   "train": f"{args.ws_train} instances L=1e5 n=2e4 (the L=2e6 generator at "
                            f"L=1e5), targets after {args.ws_target_iters} iterations",
                   "epochs": args.ws_epochs, "tau0": args.ws_tau0, "tau_decay": args.tau_decay,
                   "decay_every": args.decay_every, "max_iters": args.max_iters, "caps": caps},
        "speedup_by_level": {w: {f"{lv:g}": speedup(f"{lv:g}", w) for lv in levels}
                             for w in warms},
        "network": mlp,
        "collect_s": t_collect, "train_s": t_train, "loss_first": losses[0],
        "loss_last": losses[-1], "target_variance": float(Y.var()),
        "target_gap_median": float(np.median(gaps)), "eval": results,
    }
    print(json.dumps(out), flush=True)
    net.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--config", type=int, default=1, choices=[0, 1, 2])
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true",
                    help="skip the per-launch events (roofline fields become null)")
    ap.add_argument("--batched", action="store_true",
                    help="multi-period re-solves: a batch of instances solved in one persistent "
                         "launch per iteration against the same instances solved one by one")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-scale", type=float, default=1.0,
                    help="scales every instance's segment count (1.0: L log-uniform in [1e3, 1e6])")
    ap.add_argument("--tol", type=float, default=2e-2)
    ap.add_argument("--minibatch", action="store_true",
                    help="stochastic minibatch SPFOM: sampled segment-updates/s per B")
    ap.add_argument("--mb-fracs", nargs="+", default=["0.1", "0.01"],
                    help="minibatch mode: B as fractions of L")
    ap.add_argument("--gosim", action="store_true",
                    help="the GO bid-price policy simulation on the market of Figure 4")
    ap.add_argument("--gs-runs", type=int, default=30)
    ap.add_argument("--gs-periods", type=int, default=100)
    ap.add_argument("--gs-customers", type=int, default=1000)
    ap.add_argument("--gs-products", type=int, default=40)
    ap.add_argument("--gs-k", type=int, default=2)
    ap.add_argument("--gs-tol", type=float, default=1e-2)
    ap.add_argument("--gs-max-iters", type=int, default=1000)
    ap.add_argument("--gs-tau0", type=float, default=0.03)
    ap.add_argument("--gs-rule", default="const", choices=["const", "polyak"])
    ap.add_argument("--gs-decay", type=float, default=0.7)
    ap.add_argument("--gs-decay-every", type=int, default=100)
    ap.add_argument("--gs-persistent", type=int, default=-1, choices=[-1, 0, 1],
                    help="batched solves: -1 library default, 0 per-iteration launches, "
                         "1 one launch per solve")
    ap.add_argument("--recover", action="store_true",
                    help="time the SBLP -> CBLP recovery of one pass's sales")
    ap.add_argument("--levels", nargs="+", default=["1e-2", "3e-3", "1e-3"],
                    help="batched mode: the certified gap levels timed")
    ap.add_argument("--max-iters", type=int, default=2000)
    ap.add_argument("--warmstart", action="store_true",
                    help="learned warm start: train on solved L=1e5 instances, compare warm and "
                         "cold starts on held-out L=2e6 instances")
    ap.add_argument("--ws-caps", default="tight", choices=["tight", "loose"],
                    help="capacities 0.2-0.5x (tight, the L=2e6 workload's) or 0.5-3x (loose) "
                         "of the full-offer demand")
    ap.add_argument("--ws-train", type=int, default=512)
    ap.add_argument("--ws-target-iters", type=int, default=4000)
    ap.add_argument("--ws-epochs", type=int, default=30)
    ap.add_argument("--ws-tau0", type=float, default=3e-3)
    ap.add_argument("--ws-warm-tau", type=float, nargs="+", default=[0.1],
                    help="warm solves: their steps as multiples of tau0")
    ap.add_argument("--ws-cold-tau", type=float, nargs="+", default=[1.0, 0.3, 0.1],
                    help="cold solves: their steps as multiples of tau0")
    ap.add_argument("--ws-eval-seeds", type=int, nargs="+", default=[101, 102])
    ap.add_argument("--shuffle-products", action="store_true",
                    help="number the products in random order (the generator numbers them by "
                         "popularity; the library renumbers them by degree)")
    ap.add_argument("--oracle-seconds", type=float, default=13.0,
                    help="about how long the single-threaded oracle leg runs (whole iterations "
                         "over the whole instance, at least one)")
    ap.add_argument("--time-to-gap", action="store_true",
                    help="plain cold start: wall time and iterations to each certified gap "
                         "level (with --warmstart / --batched for the other starts)")
    ap.add_argument("--tau0", type=float, default=3e-3,
                    help="step scale: tau_i = tau0 max_j r_j / c_i")
    ap.add_argument("--tau-decay", type=float, default=0.7)
    ap.add_argument("--decay-every", type=int, default=1000)
    ap.add_argument("--bounds", nargs="+", default=["global", "segment"],
                    choices=["global", "segment"])
    ap.add_argument("--gap", type=float, default=1e-3,
                    help="the level whose time is the line's value")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy: the reference kernel whose "
                         "FETCH_SIZE / WRITE_SIZE counters scale the traffic figures")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(the multi-GPU sharding is a design, not a build)", file=sys.stderr)
        sys.exit(2)

    if (args.batched or args.warmstart or args.copy_calibration or args.time_to_gap
            or args.minibatch or args.recover or args.gosim):
        import torch
        from paper_2602_22421_amd import cblp
        cblp.load()
        if not torch.cuda.is_available():
            print("bench.py needs a GPU", file=sys.stderr)
            sys.exit(1)
        torch.cuda.set_device(0)
        if args.batched:
            return batched(args)
        if args.minibatch:
            return minibatch_bench(args)
        if args.recover:
            return recover_bench(args)
        if args.gosim:
            return gosim_bench(args)
        if args.time_to_gap:
            if "--max-iters" not in sys.argv:
                args.max_iters = 20000
            return time_to_gap(args)
        if args.warmstart:
            if "--max-iters" not in sys.argv:
                args.max_iters = 12000
            return warmstart_bench(args)
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        log("copied 1 GiB five times (read 1 GiB + write 1 GiB per copy)")
        return
    return throughput(args)


def throughput(args):
    """Whole SPFOM iterations per second on one workload (the default: the
    L=2e6, n=2e4 Zipf instance, FP32 iterate, FP64 reductions).  The CPU
    legs run first, before anything touches the GPU (their worker processes
    are forked)."""
    from paper_2602_22421_amd.instances import (CONFIG_NAMES, config_instance, shuffle_products,
                                                step_scale)
    t0 = time.perf_counter()
    inst = config_instance(args.config)
    workload = CONFIG_NAMES[args.config]
    if args.shuffle_products:
        inst = shuffle_products(inst, seed=1)[0]
        workload += "-shuffled-ids"
    npdt = np.float32 if args.dtype == "f32" else np.float64
    inst = inst.cast(npdt)
    log(f"generated {workload}: L={inst.L} n={inst.n} m={inst.m} "
        f"nnz={inst.nnz} in {time.perf_counter() - t0:.1f} s")
    tau_np = step_scale(inst, 0.001).astype(npdt)

    # CPU legs: the oracle (FP64, the same dtype-rounded inputs) on the whole
    # instance for a few iterations (its duals are also the reference of the
    # GPU's error), then the same oracle in one process per core share
    cpu = cpu_all = None
    orc_eta = orc_tr = None
    oracle_iters = max(1, int(round(args.oracle_seconds * 1.2e6 / max(inst.L, 1))))
    if not args.no_cpu_baseline:
        log(f"CPU oracle: {oracle_iters} iterations over the whole instance ...")
        cpu, orc_eta, orc_tr = cpu_baseline(inst, tau_np.astype(np.float64), oracle_iters)
        log(f"cpu baseline {cpu['value']:.3e} segment-updates/s ({cpu['sample']})")
        workers = max(1, min(16, os.cpu_count() or 1))
        reps = max(1, oracle_iters * workers // 2)
        log(f"CPU oracle on {workers} processes, {reps} iterations each over its share ...")
        cpu_all = cpu_baseline_all_cores(inst, tau_np.astype(np.float64), reps, workers)
        log(f"all-core baseline {cpu_all['value']:.3e} segment-updates/s ({cpu_all['sample']})")

    import torch
    from paper_2602_22421_amd import cblp
    cblp.load()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    dt = torch.float32 if args.dtype == "f32" else torch.float64
    prob = cblp.Problem(inst, dtype=dt)
    tau = prob.tensor(tau_np)
    params = cblp.make_params(rule=cblp.SPFOM_STEP_CONST, tau_vec=tau, check_every=10)

    # the GPU's error against the oracle at the same iteration, from eta = 0
    err = None
    if orc_eta is not None:
        e0 = prob.zeros_eta()
        trg, _ = prob.iterate(e0, oracle_iters, params)
        eg = e0.double().cpu().numpy()
        err = {"iterations": oracle_iters,
               "eta_rel_l2": float(np.linalg.norm(eg - orc_eta) / max(np.linalg.norm(orc_eta), 1e-300)),
               "eta_max_abs_over_max": float(np.max(np.abs(eg - orc_eta)) /
                                            max(np.max(np.abs(orc_eta)), 1e-300)),
               "dual_bound_rel": float(abs(trg[-1, 0] - orc_tr[-1, 0]) / abs(orc_tr[-1, 0])),
               "primal_rel": float(abs(trg[-1, 1] - orc_tr[-1, 1]) /
                                   max(abs(orc_tr[-1, 1]), 1e-300)),
               "reference": "FP64 CPU oracle on the same dtype-rounded inputs"}
        log(f"error vs oracle after {oracle_iters} iterations: {err}")
        prob.reset()

    eta = prob.zeros_eta()
    cblp.spfom_iterate(prob.h, eta, params, args.warmup)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} steps done")

    # the timed steps run without per-kernel events (they cost a few us per
    # launch); the kernel averages come from a separate instrumented run
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cblp.spfom_iterate(prob.h, eta, params, args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"timed {args.steps} steps: {wall * 1e3 / args.steps:.3f} ms/step")
    roof = None
    launch = cblp.cblp_launch_info(prob.h)
    if not args.no_timing:
        cblp.cblp_timing(prob.h, True)
        cblp.spfom_iterate(prob.h, eta, params, max(args.steps, 1))
        torch.cuda.synchronize()
        (seg_ms, dual_ms), (seg_n, dual_n) = cblp.cblp_timing_read(prob.h)
        cblp.cblp_timing(prob.h, False)
        esz = 4 if args.dtype == "f32" else 8
        nbytes, per = algorithmic_bytes(inst, esz)
        seg_avg = seg_ms / 1e3 / max(seg_n, 1)
        achieved = nbytes / seg_avg
        roof = {"bound": "hbm", "kernel": "k_segments", "achieved": achieved / 1e9,
                "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": achieved / HBM_PEAK,
                "traffic": profiled_traffic(workload) if args.dtype == "f32" else None,
                "bytes_per_launch": nbytes, "per_unit_bytes": per,
                "kernel_avg_us": seg_avg * 1e6,
                "dual_phase_avg_us": dual_ms * 1e3 / max(dual_n, 1),
                "timing": "HIP events around each launch on the launch stream, over "
                          f"{seg_n} further steps after the timed ones",
                "launch": launch}
        log(f"segment kernel {seg_avg * 1e6:.1f} us/launch, {achieved / 1e9:.0f} GB/s "
            f"({100 * achieved / HBM_PEAK:.1f}% of HBM peak); dual phase "
            f"{dual_ms * 1e3 / max(dual_n, 1):.1f} us/launch")
    st = prob.gap(eta)
    value = inst.L * args.steps / wall
    out = {
        "metric": "segment-updates/s", "value": value, "unit": "segment-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": workload, "L": inst.L, "n": inst.n,
                   "m": inst.m, "nnz": inst.nnz,
                   "iterate": args.dtype, "reductions": "f64", "step_rule": "const",
                   "dual_bound_after": st["D"]},
        "roofline": roof, "cpu_baseline": cpu, "cpu_baseline_all_cores": cpu_all,
        "error_vs_oracle": err,
    }
    print(json.dumps(out), flush=True)
    prob.close()


if __name__ == "__main__":
    main()
