"""Benchmark: SMC^2 iterations (particle-filter batch + outer step) on one MI355X.

A step is one SMC^2 iteration over the whole population: propose, N particle
filters of N_x particles over T days, L-kernel weights, normalisation, estimates,
resampling, and (learned proposal) the network's training. Default workload, the
largest that fits one GPU: the age-structured SEIR (four groups, a 4 x 4 contact
matrix, per-group negative-binomial observations of new cases), N_pop = 1e6,
T = 365, D = 8 parameters, N = 16384 parameter samples, N_x = 2048 particles,
learned proposal, FP32 propagation with FP64 log-likelihood accumulation and outer
step; synthetic observations simulated from the model at a fixed seed.

Prints one JSON line.
* value: executed particle-steps (theta x particle x day) per second of whole
  iterations, inputs resident in HBM. A filter runs N_x particles for the days up to
  the day its weights all vanish; samples with zero weight run no filter. The device
  counts what ran; the nominal N x N_x x T is reported beside it.
* roofline: the particle-filter kernel (ALU-bound): the method's algorithmic
  operations per particle-step (oracle/opcount.py) times the executed particle-steps
  of a launch, over the kernel's event-timed duration in this run, against the MI355X
  VALU peak; beside it the VALU issue rate and HBM traffic from rocprofv3 counters,
  valid while the kernel sources are those they were measured on.
* cpu_baseline: the FP64 CPU reference on a bounded sample of the workload's filters
  (the last iteration's proposals, on the GPU's random streams), at all host threads
  and at one; per executed particle-step, so extrapolated from single filters, not a
  whole iteration.
* precision: from the same reference runs, the GPU's FP32 filters against the FP64
  reference (free running; and replaying the GPU's integer decisions), and the FP64
  outer step of the last iteration against the reference recomputing it.
* ess_per_s: the metric's second part on the learned-proposal configuration (SEIR,
  D = 5, T = 150, N = 4096, N_x = 1024): recycled ESS per second at a fixed posterior
  error, learned proposal against the random walk (ess_at_fixed_error).
* secondary: the SEIR configuration (N = 1024, N_x = 512, T = 100, D = 4, RW), and the
  paper's SIR experiment, SMC^2 against p-MCMC (paper_experiment).
"""
import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Unit of work of the particle-filter kernel's roofline: algorithmic operations per
# particle-step, the reference's event counts priced by the cost table of
# oracle/opcount.py:
#   seir      python -m oracle.opcount --workload seir --N 1024 --K 12
#   age_seir  python -m oracle.opcount --workload age_seir --filters 16 --spread 0.05
# Peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 3.93e13 lane-operations/s.
ALGO_OPS_PER_PSTEP = {"seir": 647.8, "seir_learned": 647.8, "seir_batched": 647.8, "age_seir": 1393.4}
VALU_PEAK_LANE_OPS = 256 * 64 * 2.4e9
# rocprofv3 figures of the particle-filter kernel, per workload, measured on the kernel
# sources and build flags with hash `sha` (profiles/<file>): VALU instructions executed by
# active lanes per executed particle-step (SQ_INSTS_VALU x 64 x lane utilisation), HBM
# bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated on a 256 MiB device copy) and the
# VALU-busy fraction (SQ_ACTIVE_INST_VALU / 256 CUs / (GRBM_GUI_ACTIVE / 8 XCDs): cycles
# in which the VALU issued, whatever the lanes). A changed kernel reports them as null.
KERNEL_SOURCES = ["paper_2311_12973_amd/csrc/pf_kernel.hip", "paper_2311_12973_amd/csrc/pf_kernel.h",
                  "paper_2311_12973_amd/csrc/device_common.h", "paper_2311_12973_amd/csrc/block_ops.h",
                  "paper_2311_12973_amd/build.py"]
MEASURED = {
    "age_seir": dict(sha="44d6452744a009f5", valu_lane_instr_per_pstep=2397.1, hbm_bytes_per_launch=10341702729,
                     valu_busy=0.9934,
                     profile="profiles/pf_kernel_age_seir_n16384_nx2048_t365.txt"),
    "seir": dict(sha="44d6452744a009f5", valu_lane_instr_per_pstep=1416.9, hbm_bytes_per_launch=1088383,
                 valu_busy=0.9889,
                 profile="profiles/pf_kernel_seir_n1024_nx512_t100.txt"),
}


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


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


PROPOSAL_NAMES = {0: "random walk", 1: "learned proposal", 2: "Langevin proposal",
                  3: "random walk with the population's covariance"}


def describe(name, w, runs, N):
    prop = PROPOSAL_NAMES[w.get("proposal", 0)]
    prec = "FP32 propagation, FP64 accumulation and outer step" if w["prec"] == 0 else "FP64"
    if len(runs) == 1:
        return "%s N=%d Nx=%d T=%d D=%d, %s, %s" % (name, N, runs[0]["nx"], runs[0]["T"], w["D"], prop, prec)
    return "%s: %d runs, N=%d each, T in [%d, %d], Nx in %s, D=%d, %s, %s" % (
        name, len(runs), N, min(r["T"] for r in runs), max(r["T"] for r in runs), sorted({r["nx"] for r in runs}),
        w["D"], prop, prec)


def run_timed(G, W, np, name, steps, warmup, extra=0, proposal=None, **launch):
    """Build the sampler of workload `name` (with its own proposal, or `proposal`), run
    warmup + steps (+ extra untimed) iterations and time the `steps` ones. Returns the
    measurements and the sampler (open when extra > 0, after the timed steps)."""
    import torch
    w = W.preset(name)
    own_proposal = proposal is None or proposal == w.get("proposal", 0)
    if proposal is not None:
        w = dict(w, proposal=proposal)
    runs = W.batched_runs(w) if w.get("runs") else [dict(T=w["T"], nx=w["nx"], seed=w["seed"],
                                                          y=W.observations(w))]
    N = w["N"]
    s = G.Sampler(w, runs, N=N, K=warmup + steps + extra, **launch)
    for _ in range(warmup):
        s.step()
    torch.cuda.synchronize()
    s.timing()  # reset the per-iteration event timers
    ps0 = sum(int(s.dump("psteps", r)[0]) for r in range(len(runs)))
    t0 = time.perf_counter()
    for _ in range(steps):
        s.step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_pf, ms_step_dev, _ = s.timing()
    ps1 = sum(int(s.dump("psteps", r)[0]) for r in range(len(runs)))
    dead = float(np.mean([s.records(r)[warmup:warmup + steps, 3].mean() for r in range(len(runs))]))
    infos = [s.info(k) for k in range(warmup + 1, warmup + steps + 1)]
    phases = {key: float(np.mean([inf[key] for inf in infos])) for key in ("ms_filters", "ms_outer", "ms_mlp",
                                                                           "ms_step")}
    ms = (t1 - t0) * 1e3 / steps
    executed = float(ps1 - ps0)
    nominal = float(N) * sum(r["nx"] * r["T"] for r in runs) * steps
    m = dict(w=w, runs=runs, N=N, ms=ms, ms_pf=ms_pf, ms_step_dev=ms_step_dev, executed=executed, nominal=nominal,
             value=executed / ((t1 - t0)), dead=dead, steps=steps, warmup=warmup, phases=phases,
             own_proposal=own_proposal, groups=s.groups())
    if not extra:
        s.close()
        s = None
    return m, s


def roofline_of(name, m, graph):
    if graph:
        return None
    algo = ALGO_OPS_PER_PSTEP.get(name)
    launch_s = m["ms_pf"] * 1e-3
    per_launch = m["executed"] / m["steps"]
    achieved = algo * per_launch / launch_s if algo else None
    meas = MEASURED.get(name)
    # the counters were taken with the workload's own proposal (another may change the kernel)
    valid = bool(meas) and kernel_sha() == meas["sha"] and m["own_proposal"]
    issue = meas["valu_lane_instr_per_pstep"] * per_launch / launch_s if valid else None
    return {"bound": "alu", "achieved": achieved / 1e12 if algo else None, "peak": VALU_PEAK_LANE_OPS / 1e12,
            "unit": "T lane-ops/s", "frac": achieved / VALU_PEAK_LANE_OPS if algo else None,
            "traffic": meas["hbm_bytes_per_launch"] if valid else None, "kernel": "k_pf", "kernel_ms": m["ms_pf"],
            "executed_particle_steps_per_launch": per_launch,
            "algorithmic_ops_per_particle_step": algo,
            "valu_lane_instr_per_particle_step": meas["valu_lane_instr_per_pstep"] if valid else None,
            "valu_issue_frac": issue / VALU_PEAK_LANE_OPS if valid else None,
            "valu_busy": meas["valu_busy"] if valid else None,
            "profile": meas["profile"] if valid else None,
            "pf_particle_steps_per_s": per_launch / launch_s}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="age_seir")
    ap.add_argument("--graph", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--schedule", type=int, default=0, help="particle-filter draw schedule (0 auto, 1 per draw, 2 pooled)")
    ap.add_argument("--tune", type=int, default=0, help="1: time the launch configurations at init and keep the fastest")
    ap.add_argument("--persistent", type=int, default=0,
                    help="particle-filter launch: 0 automatic (a persistent grid pulling filters from the work list "
                         "when they do not fit at once), 1 persistent, 2 a workgroup per filter")
    ap.add_argument("--proposal", type=int, default=-1,
                    help="proposal of the timed workload (-1 its own; 0 random walk, 1 learned, 2 Langevin, "
                         "3 random walk with the population's covariance)")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the CPU reference leg (and the precision report)")
    ap.add_argument("--no-ess", action="store_true", help="skip the learned-proposal vs random-walk ESS/s measurement")
    ap.add_argument("--no-secondary", action="store_true", help="skip the secondary (SEIR) configuration")
    ap.add_argument("--cpu-filters", type=int, default=96, help="filters of the CPU reference sample (all threads)")
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
    launch = dict(use_graph=args.graph, block=args.block, schedule=args.schedule, tune=args.tune,
                  persistent=args.persistent)
    extra = 0 if args.no_cpu_baseline else 1
    log("workload %s: %d warm-up + %d timed iterations" % (args.workload, args.warmup, args.steps))
    m, s = run_timed(G, W, np, args.workload, args.steps, args.warmup, extra=extra,
                     proposal=args.proposal if args.proposal >= 0 else None, **launch)
    log("timed: %.1f ms per iteration, %.3g executed particle-steps/s" % (m["ms"], m["value"]))
    roofline = roofline_of(args.workload, m, args.graph)

    def section(name, fn):
        """a part of the line beside the headline: a failure is reported in the line (and on
        stderr) instead of taking the headline measurement with it"""
        try:
            return fn()
        except Exception as e:  # noqa: BLE001 - reported, not hidden
            log("%s failed: %r" % (name, e))
            return {"error": "%s: %r" % (name, e)}

    cpu = precision = None
    if s is not None:
        both = section("cpu_baseline", lambda: cpu_baseline_leg(G, np, m, s, args.cpu_filters))
        cpu, precision = (both, both) if isinstance(both, dict) else both
        s.close()

    def seir_secondary():
        m2, _ = run_timed(G, W, np, "seir", 10, 2, **launch)
        r2 = roofline_of("seir", m2, args.graph)
        log("secondary seir: %.3g particle-steps/s" % m2["value"])
        return {"workload": describe("seir", m2["w"], m2["runs"], m2["N"]), "value": m2["value"],
                "unit": "particle-steps/s", "ms_per_step": m2["ms"],
                "nominal_particle_steps_per_s": m2["nominal"] / (m2["ms"] * 1e-3 * m2["steps"]),
                "roofline_frac": r2["frac"] if r2 else None, "kernel_ms": m2["ms_pf"]}

    secondary = None
    if not args.no_secondary and args.workload != "seir":
        secondary = {"seir": section("secondary seir", seir_secondary)}

    if not args.no_secondary:
        secondary = dict(secondary or {}, paper_sir=section("paper_sir", lambda: paper_experiment(G, W, np)))

    ess = None
    if not args.no_ess:
        ess = section("ess_per_s", lambda: ess_at_fixed_error(G, W, np))

    out = {
        "metric": "PF particle-steps/s (theta x x x t), whole SMC^2 iterations; ESS/s at fixed posterior error, "
                  "learned proposal vs random walk",
        "value": m["value"], "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": m["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if m["w"]["prec"] == 0 else "f64",
        "data": "synthetic (observations simulated from the model at fixed seeds)",
        "config": {"workload": describe(args.workload, m["w"], m["runs"], m["N"]), "runs": len(m["runs"]),
                   "N": m["N"], "global_batch": m["N"] * len(m["runs"]),
                   "executed_particle_steps_per_iteration": m["executed"] / m["steps"],
                   "nominal_particle_steps_per_iteration": m["nominal"] / m["steps"],
                   "nominal_particle_steps_per_s": m["nominal"] / (m["ms"] * 1e-3 * m["steps"]),
                   "parallelism": "single GPU", "graph": bool(args.graph), "tune": bool(args.tune),
                   "persistent": any(g["persistent"] for g in m["groups"]), "dead_samples_per_step": m["dead"],
                   "device_ms_per_step": m["ms_step_dev"], "device_ms_per_phase": m["phases"],
                   "launch_groups": m["groups"]},
        "roofline": roofline, "cpu_baseline": cpu, "precision": precision, "ess_per_s": ess, "secondary": secondary,
    }
    print(json.dumps(out))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_leg(G, np, m, s, n_filters, n_single=6, n_trace=16, n_replay=256):
    """The CPU reference on a bounded sample of the workload, and what its runs say
    about the GPU's precision.

    Sample: the samples 0 .. n_filters-1 proposed in one more (untimed) iteration,
    their filters run by the FP64 reference on the GPU's random streams (filter i,
    that iteration's k) with the workload's N_x and T, on all host threads and
    (n_single of them) on one; rate = executed particle-steps (N_x x days to a
    filter's death) per second, extrapolated from single filters.
    Precision: the first n_trace of those filters traced on the GPU in FP32 (counts,
    ancestors and resampling flags of every day) against the reference's free-running
    FP64 filters (relative error of the log-likelihood; filters whose decisions differ
    anywhere, and the median day they first do) and against its FP64 replay of the
    GPU's decisions (the FP32 weight arithmetic alone); the replay alone on the first
    n_replay samples, traced in chunks of 32 (the whole-day traces are ~36 MB a filter at
    the age-structured shape); and that iteration's outer step recomputed by the
    reference from the GPU's inputs (L-kernel fit moments and log-weights)."""
    import oracle as O

    w, N, run = m["w"], m["N"], m["runs"][0]
    y, nx, T, seed = run["y"], run["nx"], run["T"], run["seed"]
    D = w["D"]
    before = {key: s.dump(key) for key in ("phi", "lp", "ll", "logw")}
    s.step()
    k = int(s.records()[-1][0])
    theta = s.dump("theta_new")
    phin, lpn, lln, lwp = (s.dump(x) for x in ("phi_new", "lp_new", "ll_new", "logw_pre"))
    used = int(s.records()[-1][G.record_len(D) - 2])  # proposal of the iteration (record column)
    lq = s.dump("logq") if used else None
    fit = s.dump("lkfit")
    anc = s.dump("anc")
    cfg64 = O.config_from_workload(w, prec=O.PREC_FP64)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    n_filters = min(n_filters, N)
    log("cpu leg: %d reference filters on %d threads (iteration %d)" % (n_filters, threads, k))

    def ref(i):
        return O.pf_trace_full(cfg64, theta[i], y, nx, seed, i, k)

    O.events_reset()
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(ref, range(n_filters)))
    dt_all = time.perf_counter() - t0
    ps_all = O.events_get()["pstep"]
    ev = O.events_get()
    O.events_reset()
    t0 = time.perf_counter()
    for i in range(n_single):
        O.pf_loglik(cfg64, theta[i], y, nx, seed, i, k)
    dt_one = time.perf_counter() - t0
    ps_one = O.events_get()["pstep"]
    from oracle.opcount import COST
    ops_sample = sum(COST[e] * ev[e] / ev["pstep"] for e in COST) if ev["pstep"] else None
    cpu = {"value": ps_all / dt_all, "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
           "sample": "FP64 reference filters of samples 0..%d of one iteration's proposals (N_x=%d, T=%d, the GPU's "
                     "streams), %.3g executed particle-steps in %.1f s on %d threads; extrapolated per executed "
                     "particle-step, not a whole iteration" % (n_filters - 1, nx, T, ps_all, dt_all, threads),
           "one_thread": ps_one / dt_one, "cpu": cpu_model(), "nproc": os.cpu_count(),
           "algorithmic_ops_per_particle_step_of_sample": ops_sample}
    log("cpu leg: %.3g particle-steps/s on %d threads, %.3g on one" % (cpu["value"], threads, cpu["one_thread"]))

    # FP32 GPU filters of the first n_trace samples with their decisions, same streams
    n_trace = min(n_trace, n_filters)
    ll32, _, rs, st, anc_t = G.pf_trace_state(w, theta[:n_trace], y, nx, seed, k, precision=G.PREC_FP32,
                                               with_anc=True)
    free, rep, differ, first = [], [], 0, []
    for i in range(n_trace):
        ll64, _, rs64, st64, anc64 = res[i]
        r64, _ = O.pf_replay(cfg64, theta[i], y, st[i], anc_t[i], rs[i])
        if np.isfinite(ll32[i]) and np.isfinite(r64):
            rep.append(abs(ll32[i] - r64) / abs(r64))
        if np.isfinite(ll32[i]) and np.isfinite(ll64):
            free.append(abs(ll32[i] - ll64) / abs(ll64))
            fd = T
            for t in range(T):
                if (rs64[t] != rs[i][t] or not np.array_equal(st64[t], st[i][t])
                        or (rs[i][t] and not np.array_equal(anc64[t], anc_t[i][t]))):
                    fd = t
                    break
            differ += fd < T
            first.append(fd + 1)
        elif np.isfinite(ll32[i]) != np.isfinite(ll64):
            differ += 1
    del st, anc_t

    # the replay on a larger sample, chunk by chunk (each replay needs only the GPU's trace)
    n_replay = min(n_replay, N)
    rep_all = []
    for c0 in range(0, n_replay, 32):
        c1 = min(c0 + 32, n_replay)
        llc, _, rsc, stc, ancc = G.pf_trace_state(w, theta[c0:c1], y, nx, seed, k, precision=G.PREC_FP32,
                                                  with_anc=True)

        def replay(i, llc=llc, rsc=rsc, stc=stc, ancc=ancc, c0=c0):
            r64, _ = O.pf_replay(cfg64, theta[c0 + i], y, stc[i], ancc[i], rsc[i])
            return abs(llc[i] - r64) / abs(r64) if np.isfinite(llc[i]) and np.isfinite(r64) else None

        with cf.ThreadPoolExecutor(threads) as ex:
            rep_all += [v for v in ex.map(replay, range(c1 - c0)) if v is not None]
        del stc, ancc
    log("precision: %d filters replayed, largest relative error %s" % (len(rep_all), max(rep_all) if rep_all else None))

    # the outer step of this iteration from the GPU's inputs
    om = np.exp(before["logw"] - np.max(before["logw"]))
    om /= om.sum()
    _, mu, cov = O.lkernel_fit_cov(before["phi"], phin, om)
    st_, lwp_ref, anc_ref, _ = O.outer_update(O.config_from_workload(w), k, seed, dict(before), phin, lpn, lln, lq)
    fin = np.isfinite(lwp_ref)
    D2 = 2 * D
    q = lambda a: None if len(a) == 0 else float(np.median(a))
    precision = {
        "filters_fp32_vs_fp64_reference": {
            "filters": n_trace, "compared": len(free),
            "free_running_rel_err_median": q(free), "free_running_rel_err_max": max(free) if free else None,
            "decisions_differ_fraction": differ / n_trace,
            "first_differing_day_median": q(first), "days": T,
            "replayed_rel_err_median": q(rep), "replayed_rel_err_max": max(rep) if rep else None,
            "replay": "FP64 reference weights on the GPU's own counts, ancestors and resampling flags"},
        "replay_sample": {
            "filters": n_replay, "compared": len(rep_all), "replayed_rel_err_median": q(rep_all),
            "replayed_rel_err_max": float(max(rep_all)) if rep_all else None,
            "within_1e-4": bool(rep_all) and bool(max(rep_all) <= 1e-4),
            "replay": "the first filters of the same iteration, each traced on the GPU (FP32) and its weights "
                      "recomputed in FP64 by the reference on the GPU's decisions"},
        "outer_fp64_vs_reference": {
            "iteration": k, "proposal": PROPOSAL_NAMES[used],
            "lkernel_mean_rel_err_max": float(np.max(np.abs(fit[:D2] - mu) / np.maximum(np.abs(mu), 1e-300))),
            "lkernel_cov_err_max_rel_to_largest": float(np.max(np.abs(fit[D2:].reshape(D2, D2) - cov))
                                                         / np.max(np.abs(cov))),
            "logw_rel_err_max": float(np.max(np.abs(lwp[fin] - lwp_ref[fin]) / np.maximum(np.abs(lwp_ref[fin]), 1)))
            if fin.any() else None,
            "zero_weights_agree": bool(np.array_equal(np.isfinite(lwp), fin)),
            "ancestors_identical": bool(np.array_equal(anc, anc_ref))},
    }
    log("precision: replayed rel err max %s, outer log-weights %s" % (
        precision["filters_fp32_vs_fp64_reference"]["replayed_rel_err_max"],
        precision["outer_fp64_vs_reference"]["logw_rel_err_max"]))
    return cpu, precision


def paper_experiment(G, W, np, seed=1):
    """The paper's SIR experiment (Sec. V, Table II: beta = 0.85, gamma = 0.2, T = 30,
    N_pop = 1e4, N_x = 500, FP64) on one MI355X, on synthetic data of that model: SMC^2
    with N = 1024 and K = 10 against p-MCMC with M = K N = 10240 samples, half burned in,
    as one chain (the paper's sequential form) and as 64 chains of 160 iterations (80
    burned in), each chain's filter in one launch per iteration. Wall time of the
    iterations (synchronised), the estimates and their squared error against the truth;
    Table II's MSE (per-run squared errors averaged over 10 runs and both parameters) for
    SMC^2 and for 64-chain p-MCMC; the analogues of Fig. 3 (the estimates per iteration)
    and Fig. 1 (the run time of K = 10 iterations for N = 256 .. 16384); the paper's
    figures (128 CPU cores for SMC^2, one for p-MCMC) beside them as context."""
    import torch
    w = W.preset("paper_sir")
    y = W.observations(w)
    truth = np.array(w["truth"])
    run = dict(T=y.shape[0], nx=w["nx"], seed=seed, y=y)
    out = {"workload": "paper_sir: SIR, T=30, N_pop=1e4, N_x=500, FP64; SMC^2 N=1024 K=10; p-MCMC M=10240"}
    s = G.Sampler(w, [run], N=w["N"], K=w["K"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(w["K"]):
        s.step()
    mean, _ = s.estimate(recycled=True)
    sec = time.perf_counter() - t0
    rec_k = s.records()
    s.close()
    out["smc2"] = {"seconds": sec, "posterior_mean": mean.tolist(), "squared_error": float(np.mean((mean - truth) ** 2))}
    # Fig. 3's analogue: the per-iteration estimates of (beta, gamma) and the recycled one
    out["smc2"]["estimates_per_iteration"] = rec_k[:, 6:8].tolist()
    # Fig. 1's analogue: the run time of K = 10 iterations against the problem size K N
    sizes = []
    for n in (256, 512, 1024, 2048, 4096, 8192, 16384):
        s = G.Sampler(w, [run], N=n, K=w["K"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(w["K"]):
            s.step()
        s.estimate(recycled=True)
        sizes.append({"N": n, "KN": n * w["K"], "seconds": time.perf_counter() - t0})
        s.close()
    out["runtime_vs_problem_size"] = sizes
    for name, chains, iters in (("pmcmc_64_chains", 64, 160), ("pmcmc_1_chain", 1, 10240)):
        mc = G.PMCMC(w, run, chains, iters)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mc.step(iters)
        m2, _, rate = mc.estimate(iters // 2)
        sec2 = time.perf_counter() - t0
        mc.close()
        out[name] = {"chains": chains, "iterations": iters, "seconds": sec2, "posterior_mean": m2.tolist(),
                     "squared_error": float(np.mean((m2 - truth) ** 2)), "acceptance": rate}
        log("paper_sir: %s %.3f s" % (name, sec2))
    # Table II's MSE: per-run squared errors averaged over 10 runs (seeds 1..10, the same data) and both
    # parameters; SMC^2 as one batched context of 10 runs, p-MCMC as 10 contexts of 64 chains
    R = 10
    s = G.Sampler(w, [dict(run, seed=r) for r in range(1, R + 1)], N=w["N"], K=w["K"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(w["K"]):
        s.step()
    means = np.array([s.estimate(r, recycled=True)[0] for r in range(R)])
    sec10 = time.perf_counter() - t0
    s.close()
    out["smc2_10_runs"] = {"runs": R, "seconds": sec10, "posterior_mean_average": means.mean(0).tolist(),
                           "mse": float(np.mean((means - truth) ** 2))}
    m64 = []
    for r in range(1, R + 1):
        mc = G.PMCMC(w, dict(run, seed=r), 64, 160)
        mc.step(160)
        m64.append(mc.estimate(80)[0])
        mc.close()
    m64 = np.array(m64)
    out["pmcmc_64_chains_10_runs"] = {"runs": R, "posterior_mean_average": m64.mean(0).tolist(),
                                      "mse": float(np.mean((m64 - truth) ** 2))}
    log("paper_sir: MSE over 10 runs, SMC^2 %.3g, p-MCMC (64 chains) %.3g"
        % (out["smc2_10_runs"]["mse"], out["pmcmc_64_chains_10_runs"]["mse"]))
    out["smc2_speedup_vs_pmcmc_1_chain"] = out["pmcmc_1_chain"]["seconds"] / out["smc2"]["seconds"]
    out["smc2_speedup_vs_pmcmc_64_chains"] = out["pmcmc_64_chains"]["seconds"] / out["smc2"]["seconds"]
    out["paper_context"] = {"smc2_seconds": 2.39, "smc2_mean": [0.8526, 0.2003], "smc2_mse": 7.75e-5,
                            "pmcmc_seconds": 130.01, "pmcmc_mean": [0.8628, 0.2038], "pmcmc_mse": 2.42e-4,
                            "hardware": "SMC^2 on 128 Xeon Gold 6138 cores, p-MCMC on one (Table II)"}
    log("paper_sir: SMC^2 %.4f s, %.1fx faster than one p-MCMC chain"
        % (out["smc2"]["seconds"], out["smc2_speedup_vs_pmcmc_1_chain"]))
    return out


def ess_at_fixed_error(G, W, np, n_ref=32768, k_ref=(30, 60), ref_seeds=3, seeds=10, k_max=(20, 60, 60, 60),
                       thresholds=(0.05, 0.1, 0.15, 0.2, 0.25, 0.3), seed0=1):
    """ESS per second at a fixed posterior error, learned proposal against the random
    walk (and, against the same random walk, the truncated Langevin proposal driven by
    the filters' score estimates and the random walk with the population's covariance),
    on the learned-proposal configuration (SEIR with the dispersion estimated, D = 5,
    T = 150, N = 4096, N_x = 1024):
    * reference posterior: `ref_seeds` long runs of each form (N = n_ref, K = k_ref;
      one batched sampler per form). Per form, f the average of its runs' recycled
      means, s the root of their average variance, and its standard error the spread
      of the runs' means over sqrt(ref_seeds), in posterior-sd units. The reference is
      the more precise of the two when the two agree within three of the other's
      standard errors on every coordinate, else the average of all runs with the
      spread of all of them; a threshold counts as resolved when it is at least twice
      the reference's largest standard error;
    * each form runs `seeds` independent runs (one batched sampler) for up to k_max
      iterations (learned, random walk, Langevin, population random walk). After
      iteration k a run's error is
      eps(k) = max_d |f_d(k) - f_ref,d| / s_ref,d, f(k) its recycled mean over
      iterations 1..k; at the first k with eps(k) <= threshold the run's ESS per second
      is its recycled ESS sum_{k' <= k} l_k' over its share of the wall time of
      iterations 1..k (the batch's time divided by the number of runs);
    * per form and threshold: the quartiles over the runs that reach it, the
      iterations taken, the runs that do not within k_max;
    * the headline: the ratio of the medians at the smallest resolved threshold that
      at least 80% of each form's runs reach; also the replicate ESS (posterior variance
      over the variance of the final recycled means across runs) per second. The
      Langevin and population random-walk forms are reported beside it, against the
      random walk at the same threshold, and the learned proposal against the population
      random walk."""
    import torch

    w = W.preset("seir_learned")
    y = W.observations(w)
    N = w["N"]
    run = lambda sd: dict(T=y.shape[0], nx=w["nx"], seed=sd, y=y)
    refs = {}
    for (name, prop), kr in zip((("learned", G.PROP_MLP), ("random_walk", G.PROP_RW)), k_ref):
        log("ess: reference, %d %s runs at N=%d, K=%d" % (ref_seeds, name, n_ref, kr))
        s = G.Sampler(dict(w, proposal=prop), [run(1000 + i) for i in range(ref_seeds)], N=n_ref, K=kr)
        t0 = time.perf_counter()
        for _ in range(kr):
            s.step()
        est = [s.estimate(r, recycled=True) for r in range(ref_seeds)]
        sec = time.perf_counter() - t0
        s.close()
        m_each = np.array([mm for mm, _ in est])
        sd = np.sqrt(np.mean([np.diag(c) for _, c in est], 0))
        refs[name] = dict(proposal=name, runs=ref_seeds, N=n_ref, K=kr, seconds=sec, each=m_each,
                          mean=m_each.mean(0), sd=sd, se=m_each.std(0, ddof=1) / np.sqrt(ref_seeds) / sd)
    a, b = refs["learned"], refs["random_walk"]
    best, other = (a, b) if a["se"].max() <= b["se"].max() else (b, a)
    agree = bool(np.all(np.abs(best["mean"] - other["mean"]) / best["sd"] <= 3 * np.maximum(other["se"], best["se"])))
    if agree:
        m_ref, s_ref, se_ref, used = best["mean"], best["sd"], best["se"], best["proposal"]
    else:
        allm = np.vstack([a["each"], b["each"]])
        s_ref = 0.5 * (a["sd"] + b["sd"])
        m_ref, se_ref, used = allm.mean(0), allm.std(0, ddof=1) / np.sqrt(len(allm)) / s_ref, "both"
    resolved = 2.0 * float(se_ref.max())
    out = {"reference": {"used": used, "forms_agree": agree, "smallest_resolved_error": resolved,
                         "posterior_mean": m_ref.tolist(), "posterior_sd": s_ref.tolist(),
                         "standard_error_in_sd": se_ref.tolist(),
                         "runs": {k: {"proposal": v["proposal"], "runs": v["runs"], "N": v["N"], "K": v["K"],
                                      "seconds": v["seconds"], "posterior_mean": v["mean"].tolist(),
                                      "standard_error_in_sd": v["se"].tolist()} for k, v in refs.items()},
                         "difference_in_sd": ((a["mean"] - b["mean"]) / s_ref).tolist()}}
    forms = (("learned", G.PROP_MLP), ("random_walk", G.PROP_RW), ("langevin", G.PROP_LANGEVIN),
             ("rw_pop", G.PROP_RW_POP))
    for (name, prop), kmax in zip(forms, k_max):
        log("ess: %s, %d runs at N=%d, up to K=%d" % (name, seeds, N, kmax))
        s = G.Sampler(dict(w, proposal=prop), [run(sd) for sd in range(seed0, seed0 + seeds)], N=N, K=kmax)
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
        est = [s.estimate(r, recycled=True) for r in range(seeds)]
        s.close()
        fm = np.array([mm for mm, _ in est])
        post_var = np.mean([np.diag(c) for _, c in est], 0)
        rep_ess = 1.0 / float(np.mean(fm.var(0, ddof=1) / post_var))
        res = {"runs": seeds, "N": N, "k_max": kmax, "iterations_run": k, "seconds": t_cum,
               "final_mean_error_in_sd": (np.mean([(mm - m_ref) / s_ref for mm in means], 0)).tolist(),
               "replicate_ess": rep_ess, "replicate_ess_per_s_per_run": rep_ess / (t_cum / seeds)}
        for th in thresholds:
            ok = np.array([x for x in rate[th] if x is not None])
            qv = np.percentile(ok, [25, 50, 75]).tolist() if len(ok) else [None] * 3
            res["eps_%g" % th] = {"iterations_to_error": first[th], "not_reached": int(sum(x is None for x in first[th])),
                                  "ess_per_s_quartiles": qv}
        out[name] = res
    head = None
    for th in thresholds:
        a = out["learned"]["eps_%g" % th]
        b = out["random_walk"]["eps_%g" % th]
        ratio = (a["ess_per_s_quartiles"][1] / b["ess_per_s_quartiles"][1]
                 if a["ess_per_s_quartiles"][1] and b["ess_per_s_quartiles"][1] else None)
        out["ratio_of_medians_eps_%g" % th] = ratio
        if (head is None and th >= resolved and ratio is not None and a["not_reached"] <= 0.2 * seeds
                and b["not_reached"] <= 0.2 * seeds):
            head = th
    out["fixed_error"] = head
    out["speedup"] = out["ratio_of_medians_eps_%g" % head] if head is not None else None
    out["replicate_ess_speedup"] = (out["learned"]["replicate_ess_per_s_per_run"] /
                                    out["random_walk"]["replicate_ess_per_s_per_run"])
    for form, against in (("langevin", "random_walk"), ("rw_pop", "random_walk"), ("learned", "rw_pop")):
        if form not in out or against not in out:
            continue
        tag = form if against == "random_walk" else "%s_vs_%s" % (form, against)
        for th in thresholds:
            a = out[form]["eps_%g" % th]
            b = out[against]["eps_%g" % th]
            out["%s_ratio_of_medians_eps_%g" % (tag, th)] = (
                a["ess_per_s_quartiles"][1] / b["ess_per_s_quartiles"][1]
                if a["ess_per_s_quartiles"][1] and b["ess_per_s_quartiles"][1] else None)
        ok = (head is not None and out[form]["eps_%g" % head]["not_reached"] <= 0.2 * seeds
              and out[against]["eps_%g" % head]["not_reached"] <= 0.2 * seeds)
        out["%s_speedup" % tag] = out["%s_ratio_of_medians_eps_%g" % (tag, head)] if ok else None
        out["%s_replicate_ess_speedup" % tag] = (out[form]["replicate_ess_per_s_per_run"] /
                                                 out[against]["replicate_ess_per_s_per_run"])
    out["protocol"] = ("recycled ESS per second at the first iteration with max_d |mean - ref| / sd_ref <= eps; "
                       "reference: %d runs of each form at N=%d (K=%d learned, %d random walk), the more precise "
                       "when they agree; %d runs per form at N=%d; speedup at the smallest resolved eps that 80%% "
                       "of each form's runs reach" % (ref_seeds, n_ref, k_ref[0], k_ref[1], seeds, N))
    out["workload"] = "seir_learned: D=5, T=150, N=4096, N_x=1024"
    log("ess: speedup %s at eps %s (replicate ESS %.3g); Langevin %s (replicate ESS %.3g); population random "
        "walk %s (replicate ESS %.3g); learned against it %s (replicate ESS %.3g)"
        % (out["speedup"], head, out["replicate_ess_speedup"], out.get("langevin_speedup"),
           out.get("langevin_replicate_ess_speedup", float("nan")), out.get("rw_pop_speedup"),
           out.get("rw_pop_replicate_ess_speedup", float("nan")), out.get("learned_vs_rw_pop_speedup"),
           out.get("learned_vs_rw_pop_replicate_ess_speedup", float("nan"))))
    return out


if __name__ == "__main__":
    main()
