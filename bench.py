"""Benchmark: SMC^2 iterations (particle-filter batch + outer step) on one MI355X.

A step is one SMC^2 iteration over the whole population: propose, N particle
filters of N_x particles over T days, L-kernel weights, normalisation, estimates,
resampling. Workload (default): SEIR, N_pop = 1e6, negative-binomial observations of
new cases, T = 100, D = 4, N = 1024 parameter samples, N_x = 512 particles, FP32
propagation with FP64 log-likelihood and outer step; synthetic observations
simulated from a fixed seed.

Prints one JSON line. value = particle-steps per second (theta x particle x day)
of whole iterations, inputs resident in HBM. roofline: the particle-filter kernel
(ALU-bound) -- algorithmic operations per second (the method's operation count per
particle-step times the particle-steps of a launch, over the kernel's event-timed
duration in this run) against the MI355X VALU peak; beside it the VALU issue rate
the kernel actually sustains, from its rocprofv3 instruction counts.
cpu_baseline: the CPU reference on a bounded sample of the same workload.
ess_per_s: the metric's second part -- ESS per second at the same posterior, learned
proposal against the random walk (see ess_per_second).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Roofline of the particle-filter kernel: ALU-bound (counts and log-weights stay on
# chip; its algorithmic HBM traffic is theta, y and one log-likelihood per filter).
# Unit of work: algorithmic operations per particle-step -- the reference sampler's
# event counts on this workload (whole run, N = 1024, K = 12) priced by the cost table
# of oracle/opcount.py (`python -m oracle.opcount --workload seir --N 1024 --K 12`).
# Peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 3.93e13 lane-operations/s.
ALGO_OPS_PER_PSTEP = {"seir": 708.8}
VALU_PEAK_LANE_OPS = 256 * 64 * 2.4e9
# Measured on the kernel sources and build flags with hash KERNEL_SHA (rocprofv3 passes recorded in
# profiles/pf_kernel_seir_n1024_nx512_t100.txt, default workload and launch): VALU
# instructions executed by active lanes per particle-step (SQ_INSTS_VALU x 64 x VALU
# utilisation / particle-steps) and HBM bytes per launch (FETCH_SIZE / WRITE_SIZE,
# calibrated on a 256 MiB device copy). Changed sources report them as null.
KERNEL_SOURCES = ["paper_2311_12973_amd/csrc/pf_kernel.hip", "paper_2311_12973_amd/csrc/pf_kernel.h",
                  "paper_2311_12973_amd/csrc/device_common.h", "paper_2311_12973_amd/csrc/block_ops.h",
                  "paper_2311_12973_amd/build.py"]
KERNEL_SHA = "35952fdc1a70dab8"
PROFILED_WORKLOAD = "seir"
VALU_LANE_INSTR_PER_PSTEP = 1427.3
HBM_BYTES_PER_LAUNCH = 1.0342e6


def kernel_sha():
    """Hash of the kernel sources and build flags with comments and whitespace removed
    (a documentation edit leaves it unchanged)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f)) as fh:
            text = fh.read()
        if f.endswith(".py"):
            text = re.sub(r"#[^\n]*", "", text)
        else:
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            text = re.sub(r"//[^\n]*", "", text)
        h.update(re.sub(r"\s+", "", text).encode())
    return h.hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="seir")
    ap.add_argument("--graph", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--schedule", type=int, default=0, help="particle-filter draw schedule (0 auto, 1 per draw, 2 pooled)")
    ap.add_argument("--tune", type=int, default=0, help="1: time the launch configurations at init and keep the fastest")
    ap.add_argument("--persistent", type=int, default=0, help="1: persistent grid pulling filters from the work list")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ess", action="store_true", help="skip the learned-proposal vs random-walk ESS/s comparison")
    ap.add_argument("--ess-protocol", type=int, default=0,
                    help="1: ESS/s at a fixed posterior error against a long reference run (about a minute more)")
    ap.add_argument("--ess-protocol-n", type=int, default=0, help="samples per run of that protocol (0: the workload's)")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB before the timed region (calibrates "
                         "the FETCH_SIZE / WRITE_SIZE counters of a profiling run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the sampler runs on one GPU (it is not sharded across GPUs); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2311_12973_amd as G
    from paper_2311_12973_amd import workloads as W

    torch.cuda.set_device(0)
    if args.copy_calib_mb:
        src = torch.ones(args.copy_calib_mb << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = W.preset(args.workload)
    if w.get("runs"):
        runs = W.batched_runs(w)
    else:
        runs = [dict(T=w["T"], nx=w["nx"], seed=w["seed"], y=W.observations(w))]
    N = w["N"]
    K = args.warmup + args.steps
    s = G.Sampler(w, runs, N=N, K=K, use_graph=args.graph, block=args.block, schedule=args.schedule, tune=args.tune,
                  persistent=args.persistent)
    for _ in range(args.warmup):
        s.step()
    torch.cuda.synchronize()
    s.timing()  # reset the per-iteration event timers
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s.step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_pf, ms_step_dev, n_timed = s.timing()
    dead = float(np.mean([s.records(r)[args.warmup:, 3].mean() for r in range(len(runs))]))
    s.close()

    ms = (t1 - t0) * 1e3 / args.steps
    psteps = float(N) * sum(r["nx"] * r["T"] for r in runs)
    value = psteps / (ms * 1e-3)

    roofline = None
    if not args.graph:
        launch_s = ms_pf * 1e-3
        algo = ALGO_OPS_PER_PSTEP.get(args.workload)
        achieved = algo * psteps / launch_s if algo else None
        measured = kernel_sha() == KERNEL_SHA and args.workload == PROFILED_WORKLOAD and args.schedule == 0
        issue = VALU_LANE_INSTR_PER_PSTEP * psteps / launch_s if measured else None
        roofline = {"bound": "alu", "achieved": achieved / 1e12 if algo else None,
                    "peak": VALU_PEAK_LANE_OPS / 1e12, "unit": "T lane-ops/s",
                    "frac": achieved / VALU_PEAK_LANE_OPS if algo else None,
                    "traffic": HBM_BYTES_PER_LAUNCH if measured else None,
                    "kernel": "k_pf", "kernel_ms": ms_pf, "algorithmic_ops_per_particle_step": algo,
                    "valu_lane_instr_per_particle_step": VALU_LANE_INSTR_PER_PSTEP if measured else None,
                    "valu_issue_frac": issue / VALU_PEAK_LANE_OPS if measured else None,
                    "pf_particle_steps_per_s": psteps / launch_s}

    ess = None
    if not args.no_ess:
        ess = ess_per_second(G, W, np)
        if args.ess_protocol:
            ess["at_fixed_error"] = ess_at_fixed_error(G, W, np, n_runs=args.ess_protocol_n or None)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, runs)
    if len(runs) == 1:
        desc = "%s N=%d Nx=%d T=%d D=%d %s propagation, FP64 outer" % (
            args.workload, N, runs[0]["nx"], runs[0]["T"], w["D"], "FP32" if w["prec"] == 0 else "FP64")
    else:
        desc = "%s: %d runs, N=%d each, T in [%d, %d], Nx in %s, D=%d %s propagation, FP64 outer" % (
            args.workload, len(runs), N, min(r["T"] for r in runs), max(r["T"] for r in runs),
            sorted({r["nx"] for r in runs}), w["D"], "FP32" if w["prec"] == 0 else "FP64")

    out = {
        "metric": "PF particle-steps/s (theta x x x t), whole SMC^2 iterations",
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32" if w["prec"] == 0 else "f64",
        "data": "synthetic (observations simulated from the model at fixed seeds)",
        "config": {"workload": desc, "runs": len(runs), "N": N, "global_batch": N * len(runs),
                   "particle_steps_per_iteration": psteps, "parallelism": "single GPU", "graph": bool(args.graph),
                   "tune": bool(args.tune), "persistent": bool(args.persistent),
                   "dead_samples_per_step": dead, "device_ms_per_step": ms_step_dev},
        "roofline": roofline, "cpu_baseline": cpu, "ess_per_s": ess,
    }
    print(json.dumps(out))


def ess_per_second(G, W, np):
    """ESS per second at the same posterior, learned proposal vs random walk, on the
    learned-proposal configuration: SEIR with the dispersion estimated (D = 5), T = 150,
    N = 4096, N_x = 1024, K = 20; 16 independent runs of each form (one batched sampler
    per form). Replicate ESS = posterior variance / variance of the recycled posterior
    mean across runs (averaged over coordinates); per second of the whole batch's
    iterations, per run. The variance across R runs has a relative standard error of
    about sqrt(2 / (R - 1)), reported with it. Also the recycled ESS sum_k l_k of each
    run per second."""
    import torch

    w = W.preset("seir_learned")
    y = W.observations(w)
    seeds = list(range(1, 17))
    K = w["K"]
    out = {}
    for name, prop in (("learned", G.PROP_MLP), ("random_walk", G.PROP_RW)):
        s = G.Sampler(dict(w, proposal=prop), [dict(T=y.shape[0], nx=w["nx"], seed=sd, y=y) for sd in seeds],
                      N=w["N"], K=K)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(K):
            s.step()
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        est = [s.estimate(r, recycled=True) for r in range(len(seeds))]
        wess = float(np.mean([s.records(r)[1:, 1].mean() for r in range(len(seeds))]))
        ress = float(np.mean([s.records(r)[:, 1].sum() for r in range(len(seeds))]))  # recycled ESS, sum_k l_k
        s.close()
        means = np.array([m for m, _ in est])
        post_var = np.mean([np.diag(c) for _, c in est], 0)
        ess = 1.0 / float(np.mean(means.var(0, ddof=1) / post_var))
        out[name] = {"N": w["N"], "replicate_ess": ess, "weight_ess_per_iteration": wess, "seconds": sec,
                     "recycled_ess": ress, "recycled_ess_per_s_per_run": ress / (sec / len(seeds)),
                     "ess_per_s_per_run": ess / (sec / len(seeds)), "posterior_mean": means.mean(0).tolist(),
                     "posterior_sd": np.sqrt(post_var).tolist()}
    sd = 0.5 * (np.array(out["learned"]["posterior_sd"]) + np.array(out["random_walk"]["posterior_sd"]))
    out["mean_difference_in_sd"] = ((np.array(out["learned"]["posterior_mean"]) -
                                     np.array(out["random_walk"]["posterior_mean"])) / sd).tolist()
    out["speedup"] = out["learned"]["ess_per_s_per_run"] / out["random_walk"]["ess_per_s_per_run"]
    out["recycled_ess_speedup"] = (out["learned"]["recycled_ess_per_s_per_run"] /
                                   out["random_walk"]["recycled_ess_per_s_per_run"])
    out["replicate_ess_rel_se"] = float(np.sqrt(2.0 / (len(seeds) - 1)))
    out["workload"] = "seir_learned: D=5, T=150, N=4096, N_x=1024, K=20, %d runs per form" % len(seeds)
    return out


def ess_at_fixed_error(G, W, np, n_ref=32768, k_ref=100, ref_seeds=3, seeds=10, k_max=(20, 80), n_runs=None,
                       thresholds=(0.1, 0.25)):
    """ESS per second at a fixed posterior error, learned proposal against the random
    walk, on the learned-proposal configuration (SEIR with the dispersion estimated,
    D = 5, T = 150, N = 4096, N_x = 1024):
    * reference posterior: `ref_seeds` long random-walk runs (N = n_ref, K = k_ref, one
      batched sampler), f_ref the average of their recycled means and s_ref the root of
      their average variance; the reference's own standard error, the spread of the
      runs' means over sqrt(ref_seeds), is reported in s_ref units;
    * each form runs `seeds` independent runs (one batched sampler) for up to k_max
      iterations (learned, random walk). After iteration k a run's error is
      eps(k) = max_d |f_d(k) - f_ref,d| / s_ref,d, f(k) its recycled mean over
      iterations 1..k; at the first k with eps(k) <= threshold the run's ESS per second
      is its recycled ESS sum_{k' <= k} l_k' over its share of the wall time of
      iterations 1..k (the batch's time divided by the number of runs);
    * reported per form and threshold: the median and quartiles over the runs that
      reach it, the iterations taken and the runs that do not within k_max; the mean
      error of the final means per coordinate (in s_ref units); and the ratio of medians."""
    import torch

    w = W.preset("seir_learned")
    y = W.observations(w)
    N = n_runs or w["N"]
    run = lambda sd: dict(T=y.shape[0], nx=w["nx"], seed=sd, y=y)
    s = G.Sampler(dict(w, proposal=G.PROP_RW), [run(1000 + i) for i in range(ref_seeds)], N=n_ref, K=k_ref)
    t0 = time.perf_counter()
    for _ in range(k_ref):
        s.step()
    ref = [s.estimate(r, recycled=True) for r in range(ref_seeds)]
    t_ref = time.perf_counter() - t0
    s.close()
    m_each = np.array([m for m, _ in ref])
    m_ref = m_each.mean(0)
    s_ref = np.sqrt(np.mean([np.diag(c) for _, c in ref], 0))
    se_ref = m_each.std(0, ddof=1) / np.sqrt(ref_seeds) / s_ref if ref_seeds > 1 else np.full(len(m_ref), np.nan)
    out = {"reference": {"proposal": "random walk", "runs": ref_seeds, "N": n_ref, "K": k_ref, "seconds": t_ref,
                         "posterior_mean": m_ref.tolist(), "posterior_sd": s_ref.tolist(),
                         "standard_error_in_sd": se_ref.tolist(),
                         "run_means_in_sd": ((m_each - m_ref) / s_ref).tolist()}}
    for (name, prop), kmax in zip((("learned", G.PROP_MLP), ("random_walk", G.PROP_RW)), k_max):
        s = G.Sampler(dict(w, proposal=prop), [run(sd) for sd in range(1, seeds + 1)], N=N, K=kmax)
        t_cum = 0.0
        first = {th: [None] * seeds for th in thresholds}
        rate = {th: [None] * seeds for th in thresholds}
        for k in range(1, kmax + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.step()
            torch.cuda.synchronize()
            t_cum += time.perf_counter() - t0
            means = [s.estimate(r, recycled=True)[0] for r in range(seeds)]
            for r in range(seeds):
                eps = float(np.max(np.abs(means[r] - m_ref) / s_ref))
                for th in thresholds:
                    if first[th][r] is None and eps <= th:
                        first[th][r] = k
                        rate[th][r] = float(s.records(r)[:k, 1].sum()) / (t_cum / seeds)
            if all(x is not None for x in first[min(thresholds)]):
                break
        s.close()
        res = {"runs": seeds, "N": N, "k_max": kmax, "iterations_run": k,
               "final_mean_error_in_sd": (np.mean([(m - m_ref) / s_ref for m in means], 0)).tolist()}
        for th in thresholds:
            ok = np.array([x for x in rate[th] if x is not None])
            q = np.percentile(ok, [25, 50, 75]).tolist() if len(ok) else [None] * 3
            res["eps_%g" % th] = {"iterations_to_error": first[th], "not_reached": int(sum(x is None for x in first[th])),
                                  "ess_per_s_quartiles": q}
        out[name] = res
    for th in thresholds:
        a = out["learned"]["eps_%g" % th]["ess_per_s_quartiles"][1]
        b = out["random_walk"]["eps_%g" % th]["ess_per_s_quartiles"][1]
        out["ratio_of_medians_eps_%g" % th] = a / b if a and b else None
    out["protocol"] = ("recycled ESS per second at the first iteration with max_d |mean - ref| / sd_ref <= eps; "
                       "reference: %d random-walk runs, N=%d, K=%d; %d runs per form at N=%d"
                       % (ref_seeds, n_ref, k_ref, seeds, N))
    return out


def cpu_baseline(w, runs):
    """The CPU reference (all host threads) on a bounded sample of the same workload:
    the full population of N parameter samples for the first SMC^2 iterations of the
    first run(s), about ten seconds of work."""
    import oracle as O

    cfg = O.config_from_workload(w)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    n_sample = w["N"]
    k_sample = 6 if len(runs) == 1 else 2
    sample = runs[:1] if len(runs) == 1 else runs[:8]
    t = time.perf_counter()
    for r in sample:
        O.smc2_run(cfg, r["y"], r["nx"], r["seed"], n_sample, k_sample, n_threads=threads)
    dt = time.perf_counter() - t
    ps = float(n_sample) * k_sample * sum(r["nx"] * r["T"] for r in sample)
    return {"value": ps / dt, "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
            "sample": "%d run(s) of the workload, N=%d samples x %d iterations each, %.1f s"
                      % (len(sample), n_sample, k_sample, dt)}


if __name__ == "__main__":
    main()
