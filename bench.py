#!/usr/bin/env python3
"""Benchmark: energy+gradient evaluations per second of the infinite binary MERA optimisation on one MI355X.

Workload (default): TFIM h = 1 with two spins per blocked site (d = 4, 3-site term), chi = 24, three transition
layers plus the scale-invariant layer, Haar-random initial tensors (seed 2), FP32 MFMA contractions with FP64
retraction / density-matrix normalisation / L-BFGS scalars, Hilbert-space preconditioner, L-BFGS memory 8,
warm-started Krylov solves (the library's default dimension: 16 at this size). One step = one L-BFGS iteration of the library's optimiser
(mera_opt_step): its energy+gradient evaluation(s), projection, preconditioned two-loop, line search,
polar retraction and transport. value = evaluations / second over the timed steps.

Prints ONE JSON line. `--serve` instead runs a serving stream through the continuous-batching server and reports
p50/p99 time-to-converged and jobs/s.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MERA energy+gradient evals/s at chi=24 (TFLOP/s, % peak); job p50/p99 latency"
# Dense MFMA peaks in the flops the library counts (2 per multiply-add of the contraction). The split-bf16 form
# spends three bf16 products on each multiply-add, so its ceiling is a third of the 2.5 PFLOP/s bf16 peak.
PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6, "bf16x3": 2500.0 / 3}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--chi", type=int, default=24)
    ap.add_argument("--T", type=int, default=3)
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp64", "bf16x3"])
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fp64-steps", type=int, default=2,
                    help="optimiser iterations of the plain FP64 form timed for comparison (0: skip)")
    ap.add_argument("--fp64-warmup", type=int, default=1)
    ap.add_argument("--cpu-sample-chi", type=int, default=6)
    ap.add_argument("--bf16x3-steps", type=int, default=2,
                    help="optimiser iterations of the BF16X3 form timed for comparison (0: skip)")
    ap.add_argument("--serve", action="store_true")
    ap.add_argument("--jobs", type=int, default=16)
    ap.add_argument("--serve-iters", type=int, default=30)
    ap.add_argument("--serve-tol", type=float, default=1e-7, help="serving: converged at |G| <= this")
    ap.add_argument("--serve-chis", default="8,12,16,20", help="serving: bond dimensions drawn uniformly")
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--no-serve-leg", action="store_true",
                    help="skip the short serving stream reported beside the evaluation benchmark")
    ap.add_argument("--serve-leg-jobs", type=int, default=12)
    ap.add_argument("--no-group", action="store_true", help="serving: no grouped launches across jobs")
    ap.add_argument("--no-graphs", action="store_true", help="serving: no HIP graph replay")
    ap.add_argument("--max-wait-us", type=float, default=-1.0,
                    help="serving: fixed bound of a leader's wait for same-shape jobs (< 0: the library's default, "
                         "a tenth of the program's estimated run time)")
    ap.add_argument("--profile-all", action="store_true",
                    help="time every contraction launch of the run (not only the timed steps) and print the per-variant "
                         "launch counts, algorithmic flops and bytes to stderr, for comparison with a rocprofv3 trace")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (reference dispatch for hardware byte counters)")
    return ap.parse_args()


def _time_oracle_evals(params, h3, chi, T, budget_s):
    """Full oracle energy+gradient evaluations (oracle.mera.evaluate) of the same point until budget_s has passed;
    returns (evaluations, seconds)."""
    from oracle import mera as om
    t0 = time.perf_counter()
    n = 0
    while True:
        om.evaluate(params, h3, chi, T)
        n += 1
        dt = time.perf_counter() - t0
        if dt > budget_s:
            return n, dt


def cpu_baseline(a, sample_chi, sample_T, flops_sample, flops_bench):
    """The FP64 oracle's whole energy+gradient evaluation (ascending sweep, fixed point, h~, per-occurrence
    environments: oracle.mera.evaluate, as it stands) timed on the host cores at a bond dimension it finishes in
    seconds, on the benchmark's model and seed; also at the smallest configuration (chi = 4, T = 2) and on one
    thread. value = measured evaluations/s of the sample configuration. The benchmark-size figure is only an
    estimate (the sample's flop rate, with flops per evaluation from the library's counter at both sizes) and is
    reported separately."""
    from oracle import mera as om
    from paper_2007_03638_amd import api, inputs
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threadpool_limits = None
        threads = len(os.sched_getaffinity(0))
    h3 = api.h3_tfim(1.0)
    params = inputs.mera_init(a.seed, om.layer_dims(sample_chi, sample_T))
    om.evaluate(params, h3, sample_chi, sample_T)  # warm the BLAS pool
    n, dt = _time_oracle_evals(params, h3, sample_chi, sample_T, 12.0)
    rate = n / dt
    small = inputs.mera_init(0, om.layer_dims(4, 2))
    n4, dt4 = _time_oracle_evals(small, h3, 4, 2, 3.0)
    one = None
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            n1, dt1 = _time_oracle_evals(small, h3, 4, 2, 3.0)
        one = n1 / dt1
    return dict(value=rate, unit=f"evals/s (chi={sample_chi}, T={sample_T} sample)", cores=threads, kind="oracle",
                sample=f"oracle.mera.evaluate (FP64 numpy/scipy) of the benchmark's model and seed at chi={sample_chi}, "
                       f"T={sample_T}: {n} evaluations in {dt:.1f} s on {threads} BLAS threads; at chi=4, T=2: "
                       f"{n4} in {dt4:.1f} s; on 1 thread at chi=4, T=2: "
                       + (f"{one:.3g} evals/s" if one else "not measured"),
                chi4_T2_evals_per_s=n4 / dt4, one_thread_chi4_T2_evals_per_s=one,
                sample_gflops=rate * flops_sample / 1e9,
                estimate_bench_evals_per_s=rate * flops_sample / flops_bench,
                estimate_note=f"estimate for chi={a.chi}: the sample's flop rate divided by the algorithmic flops of "
                              f"one chi={a.chi} evaluation (library MAC counter: {flops_sample:.3e} flop at the sample, "
                              f"{flops_bench:.3e} at chi={a.chi})")


def counter_traffic(kernel_variant):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter summary, or None when the
    kernel source changed since the counters were taken or the summary covers another variant."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "gett_f32_chi24_counters.md")
    src = os.path.join(ROOT, "paper_2007_03638_amd", "csrc", "gett.hip")
    if not os.path.exists(path):
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    fields = dict(l.split(": ", 1) for l in open(path).read().splitlines() if ": " in l and not l.startswith("|"))
    if fields.get("gett_source_sha256_prefix", "").strip() != sha:
        return None
    if fields.get("kernel_variant", "").strip() != kernel_variant:
        return None
    return float(fields["traffic_bytes_per_launch"])


def precision_check(a, ctx, opt, h3):
    """Energy and Riemannian-gradient error of the contraction precision at the final point of the timed steps,
    against the plain FP64 evaluation of the same tensors (the FP64 GPU path, itself checked against the FP64
    oracle element by element in the parity tests)."""
    import torch
    from paper_2007_03638_amd import api
    fin = opt.final()
    u, w = fin[0::2], fin[1::2]
    r = {}
    for prec in (a.prec, "fp64"):
        ev = ctx.energy_grad(a.T, a.chi, u, w, h3, prec=prec)
        D = [x for pair in zip(ev["Du"], ev["Dw"]) for x in pair]
        W = [torch.as_tensor(x, dtype=torch.float64, device="cuda") for x in fin]
        G = ctx.stiefel_project(W, D)
        r[prec] = (ev["energy"], G)
    e_lo, G_lo = r[a.prec]
    e_hi, G_hi = r["fp64"]
    num = sum(float(torch.sum((x - y) ** 2)) for x, y in zip(G_lo, G_hi)) ** 0.5
    den = sum(float(torch.sum(y ** 2)) for y in G_hi) ** 0.5
    return {"energy": e_lo, "energy_fp64": e_hi, "energy_rel_error": abs(e_lo - e_hi) / abs(e_hi),
            "gradient_rel_error": num / den, "gnorm_fp64": den}


def form_rate(a, prec, steps, warmup):
    """Evaluations/s of another contraction precision on the same workload (same seed and start point)."""
    import torch
    from paper_2007_03638_amd import api, inputs
    ctx = api.Context(0)
    dims = api.layer_dims(a.T, a.chi)
    init = [m for pair in inputs.mera_init(a.seed, dims) for m in pair]
    opt = ctx.optimizer(T=a.T, chi=a.chi, h3=api.h3_tfim(1.0), init=init, prec=prec, m=8, max_iter=10 ** 6,
                        grad_tol=0.0, polish_tol=0.0, precondition=True, max_ls_evals=10)
    state = None
    for _ in range(warmup):
        _, state = opt.step()
    s0 = state if state is not None else {"evaluations": 1}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, state = opt.step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    evals = state["evaluations"] - s0["evaluations"]
    print(f"[bench] {prec} form: {evals} evaluations in {dt:.1f} s", file=sys.stderr, flush=True)
    return evals / dt


def run_eval_bench(a):
    import torch
    from paper_2007_03638_amd import api, inputs

    ctx = api.Context(0)
    if a.copy_calibration:
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    dims = api.layer_dims(a.T, a.chi)
    init = [m for pair in inputs.mera_init(a.seed, dims) for m in pair]
    h3 = api.h3_tfim(1.0)
    all_stats = []
    if a.profile_all:
        ctx.profile(True)
    opt = ctx.optimizer(T=a.T, chi=a.chi, h3=h3, init=init, prec=a.prec, m=8, max_iter=10 ** 6, grad_tol=0.0,
                        polish_tol=0.0, precondition=True, max_ls_evals=10)
    state = None
    for i in range(a.warmup):
        _, state = opt.step()
        print(f"[bench] warmup step {i + 1}/{a.warmup}: e={state['energy']:.12f} |G|={state['gnorm']:.3e}",
              file=sys.stderr, flush=True)
    # state after the untimed part (with no warmup: the initial evaluation done at creation)
    s0 = state if state is not None else {"evaluations": 1, "macs": ctx.macs(), "krylov_applications": 0}
    ctx.profile(True)
    all_stats += ctx.kernel_stats()  # clears the records before the timed steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        _, state = opt.step()
        print(f"[bench] step {i + 1}/{a.steps}: e={state['energy']:.12f} |G|={state['gnorm']:.3e} "
              f"evaluations={state['evaluations']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = ctx.kernel_stats()
    all_stats += stats
    ctx.profile(a.profile_all)
    dt = t1 - t0
    evals = state["evaluations"] - s0["evaluations"]
    macs = state["macs"] - s0["macs"]
    flops = 2.0 * macs
    top = stats[0]
    achieved = top["flops"] / top["seconds"] / 1e12
    gemm_time = sum(s["seconds"] for s in stats)
    peak = PEAK_TFLOPS[a.prec]
    out = {
        "metric": METRIC,
        "value": evals / dt,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1000.0 * dt / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "bf16x3": "bf16x3 (f32 accumulate)"}[a.prec],
        "data": "synthetic",
        "config": {"workload": f"infinite binary MERA, TFIM h=1 (d=4, 3-site term), chi={a.chi}, T={a.T} + "
                               f"scale-invariant layer, {a.prec} contractions, FP64 manifold/L-BFGS, "
                               f"preconditioned L-BFGS m=8, seed {a.seed}",
                   "chi": a.chi, "T": a.T, "prec": a.prec, "evaluations": evals},
        "tflops": flops / dt / 1e12,
        "pct_peak": 100.0 * flops / dt / 1e12 / peak,
        "energy": state["energy"],
        "gnorm": state["gnorm"],
        "contraction_time_fraction": gemm_time / dt,
        "roofline": {"bound": "mfma", "kernel": top["kernel"], "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": counter_traffic(top["kernel"]),
                     "algorithmic_bytes": top["bytes"] / top["launches"],
                     "launches": top["launches"], "avg_launch_ms": 1000.0 * top["seconds"] / top["launches"]},
        "krylov_applications_per_eval": (state["krylov_applications"] - s0.get("krylov_applications", 0)) / max(evals, 1),
        "kernels": [{"kernel": s["kernel"], "launches": s["launches"], "ms": 1000.0 * s["seconds"],
                     "tflops": s["flops"] / s["seconds"] / 1e12} for s in stats[:6]],
    }
    if a.prec != "fp64":
        out["precision_vs_fp64"] = precision_check(a, ctx, opt, h3)
        print(f"[bench] precision check: {out['precision_vs_fp64']}", file=sys.stderr, flush=True)
    if a.profile_all:
        all_stats += ctx.kernel_stats()
        ctx.profile(False)
        merged = {}
        for s in all_stats:
            m = merged.setdefault(s["kernel"], {"kernel": s["kernel"], "launches": 0, "seconds": 0.0, "flops": 0.0,
                                                "bytes": 0.0})
            for k in ("launches", "seconds", "flops", "bytes"):
                m[k] += s[k]
        rows = sorted(merged.values(), key=lambda m: -m["seconds"])
        for m in rows:
            m["flops_per_launch"] = m["flops"] / m["launches"]
            m["bytes_per_launch"] = m["bytes"] / m["launches"]
        print("[bench] all-launch kernel stats: " + json.dumps(rows), file=sys.stderr, flush=True)
    if a.fp64_steps > 0 and a.prec != "fp64":
        r64 = form_rate(a, "fp64", a.fp64_steps, a.fp64_warmup)
        out["fp64_form_evals_per_s"] = r64
        out["speedup_vs_fp64_form"] = out["value"] / r64
    if a.bf16x3_steps > 0 and a.prec == "fp32":
        out["bf16x3_form_evals_per_s"] = form_rate(a, "bf16x3", a.bf16x3_steps, 1)
        out["speedup_bf16x3_vs_fp32"] = out["bf16x3_form_evals_per_s"] / out["value"]
    if not a.no_cpu_baseline:
        # flops of one (cold-started, as the oracle's) FP64 evaluation at the sample size, from the library's counter
        sp = inputs.mera_init(a.seed, api.layer_dims(a.T, a.cpu_sample_chi))
        sample = ctx.energy_grad(a.T, a.cpu_sample_chi, [p[0] for p in sp], [p[1] for p in sp], h3, prec="fp64")
        out["cpu_baseline"] = cpu_baseline(a, a.cpu_sample_chi, a.T, 2.0 * sample["macs"], flops / max(evals, 1))
    return out


def run_serve_bench(a):
    """Serving stream: Poisson arrivals (mean gap 2 s, seed 3), TFIM h ~ U[0.5, 1.5] or XXZ delta ~ U[-0.5, 1.5]
    (50/50), chi from {8, 12, 16, 20} (--serve-chis), FP32 contractions with FP64 polishing, stop at |G| <= 1e-7
    (--serve-tol) or the iteration cap."""
    from paper_2007_03638_amd import api, inputs
    rng = np.random.default_rng(3)
    ctx = api.Context(0)
    srv = api.Server(ctx, hbm_budget=200 << 30, max_slots=a.slots, group_launches=not a.no_group,
                     graph_capture=not a.no_graphs, max_wait_us=None if a.max_wait_us < 0 else a.max_wait_us)
    jobs = []
    t_arr = 0.0
    for k in range(a.jobs):
        t_arr += rng.exponential(2.0)
        chi = int(rng.choice([int(c) for c in a.serve_chis.split(",")]))
        if rng.random() < 0.5:
            h3 = api.h3_tfim(rng.uniform(0.5, 1.5))
        else:
            h3 = api.h3_xxz(rng.uniform(-0.5, 1.5))
        dims = api.layer_dims(3, chi)
        init = [m for pair in inputs.mera_init(1000 + k, dims) for m in pair]
        jobs.append((t_arr, dict(T=3, chi=chi, h3=h3, init=init, prec="fp32", m=8, max_iter=a.serve_iters,
                                 grad_tol=a.serve_tol, polish_tol=1e-5)))
    t0 = time.perf_counter()
    ids, arrivals = [], []
    pending = list(jobs)
    results = {}
    while pending or len(results) < len(ids):
        now = time.perf_counter() - t0
        while pending and pending[0][0] <= now:
            arr, spec = pending.pop(0)
            ids.append(srv.submit(**spec))
            arrivals.append(arr)
        for i in ids:
            if i not in results:
                r = srv.poll(i)
                if r is not None:
                    results[i] = (time.perf_counter() - t0, r)
                    print(f"[serve] job {i} done at {results[i][0]:.1f} s: status {r['status']} "
                          f"iters {r['iterations']} |G| {r['gnorm']:.2e} latency "
                          f"{r['queued_seconds'] + r['seconds']:.1f} s ({len(results)}/{len(jobs)})",
                          file=sys.stderr, flush=True)
        time.sleep(0.005)
    makespan = time.perf_counter() - t0
    stats = srv.stats()
    srv.close()
    lat = np.array([results[i][1]["queued_seconds"] + results[i][1]["seconds"] for i in ids])
    status = np.array([results[i][1]["status"] for i in ids])
    conv = lat[status == 0]
    pct = (lambda x, q: float(np.percentile(x, q)) if len(x) else None)
    return {
        "metric": METRIC,
        "value": pct(conv, 50),
        "unit": "s (p50 time-to-converged over the converged jobs)",
        "n_gpus": 1, "steps": a.jobs, "warmup": 0,
        "ms_per_step": 1000.0 * makespan / a.jobs,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"serving stream of {a.jobs} jobs, Poisson arrivals mean gap 2 s (seed 3), TFIM/XXZ "
                               f"50/50, chi in {{{a.serve_chis}}}, T=3, FP32 + FP64 polish below 1e-5, "
                               f"stop at |G|<={a.serve_tol:g} or {a.serve_iters} iterations"},
        "converged": int(np.sum(status == 0)), "capped": int(np.sum(status == 1)),
        "failed": int(np.sum((status != 0) & (status != 1))), "iteration_cap": a.serve_iters,
        "p50_s": pct(conv, 50), "p99_s": pct(conv, 99),
        "p50_result_all_s": pct(lat, 50), "p99_result_all_s": pct(lat, 99),
        "jobs_per_s": a.jobs / makespan, "converged_per_s": float(np.sum(status == 0)) / makespan,
        "makespan_s": makespan,
        "jobs": [{"chi": jobs[k][1]["chi"], "arrival_s": arrivals[k], "status": int(results[i][1]["status"]),
                  "iterations": results[i][1]["iterations"], "gnorm": results[i][1]["gnorm"],
                  "polish_iter": results[i][1]["polish_iter"], "energy": results[i][1]["energy"],
                  "latency_s": float(lat[k])} for k, i in enumerate(ids)],
        "slots": a.slots, "grouped_launches": not a.no_group, "graph_replay": not a.no_graphs,
        "leader_wait_us": "program-cost bound" if a.max_wait_us < 0 else a.max_wait_us,
        "batcher": stats,
    }


def serve_leg(a):
    """A short converging serving stream run after the evaluation benchmark, so that its line carries measured
    job latencies: the serving stream's recipe with chi in {8, 12}, converged at |G| <= 1e-3 (a tolerance these
    jobs reach in a few hundred iterations)."""
    import copy
    b = copy.copy(a)
    b.jobs, b.serve_chis, b.serve_tol, b.serve_iters = a.serve_leg_jobs, "8,12", 1e-3, 3000
    r = run_serve_bench(b)
    keys = ("converged", "capped", "failed", "p50_s", "p99_s", "jobs_per_s", "makespan_s")
    out = {k: r[k] for k in keys}
    out["workload"] = r["config"]["workload"]
    out["unit"] = "s (time-to-converged: arrival to |G| <= 1e-3)"
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {a.gpus} is not supported: the library drives a single MI355X "
              f"and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    out = run_serve_bench(a) if a.serve else run_eval_bench(a)
    if not a.serve and not a.no_serve_leg:
        out["serving"] = serve_leg(a)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
