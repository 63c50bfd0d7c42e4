"""Benchmark of the phaseless-AFQMC step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32|bf16x3|fp64]

Workload: the large synthetic molecule-shaped Hamiltonian (M = 128 orbitals,
N = 32 + 32 electrons, N_g = 800 Cholesky vectors), 1024 walkers, dtau = 0.005,
re-orthonormalization and comb population control every 5 steps.  A step is
one full walker step (fields, force bias, propagator build, Taylor propagation,
QR when due, overlap/inverse, local-energy contraction, weights, comb when
due) for all walkers, inputs resident in HBM.  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0 / 3.0}
HBM_PEAK_GBS = 8000.0
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3"}


def eprint(*a):
    print(*a, file=sys.stderr, flush=True)


def contraction_flops(M, nup, ndn, G, n_walkers):
    """Algorithmic flops of the local-energy contraction Omega^g_s = Lh^g_s Theta_s:
    real N x M by complex M x N products, 4 G N^2 M per walker and spin."""
    return 4.0 * G * M * (nup * nup + ndn * ndn) * n_walkers


def recorded_figure(precision, name, key, cast=float):
    """A figure of the FP32 contraction from a committed counter summary under profiles/, or
    None when there is none for this precision or the kernel source changed since it was
    taken (the summary records the source's sha256)."""
    import hashlib
    if precision != "fp32":
        return None
    path = os.path.join(ROOT, "profiles", name)
    try:
        fields = dict(line.split(": ", 1) for line in open(path).read().splitlines()
                      if line.startswith((key, "kernel_source", "source_sha256")))
        src = open(os.path.join(ROOT, fields["kernel_source"].strip()), "rb").read()
        if hashlib.sha256(src).hexdigest() != fields["source_sha256"].strip():
            return None
        return cast(fields[key])
    except (OSError, KeyError, ValueError):
        return None


def recorded_traffic(precision):
    """HBM bytes per launch of the contraction (FETCH_SIZE + WRITE_SIZE, calibrated)."""
    return recorded_figure(precision, "contract_fp32_M128_N32_G800_W1024_traffic.md",
                           "traffic_bytes_per_launch", int)


def recorded_mfma_busy(precision):
    """Fraction of the contraction's active cycles the matrix cores are busy
    (SQ_VALU_MFMA_BUSY_CYCLES over GRBM_GUI_ACTIVE and the SIMDs)."""
    return recorded_figure(precision, "mfma_util_M128_N32_G800_W1024.md",
                           "mfma_busy_fp32_contraction", float)


def run_gpu(s, args, precision, steps, warmup, timed_kernels=True, closed_shell=False,
            per_step=None):
    import torch

    import paper_1711_02242_amd as afq
    gs = afq.System.from_synthetic(s, dtau=args.dtau, precision=precision, qr_period=5,
                                   pop_period=5, closed_shell=closed_shell)
    wk = gs.walkers(args.walkers)
    gs.init(wk)
    for _ in range(warmup):
        gs.step(wk, seed=args.seed)
    torch.cuda.synchronize()
    gs.bound_counts(clear=True)
    if timed_kernels:
        gs.kernel_timing(True)
    # per-step HIP events on the stream the steps run on (the current torch stream)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)] \
        if per_step is not None else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if evs:
        evs[0].record()
    for i in range(steps):
        gs.step(wk, seed=args.seed)
        if evs:
            evs[i + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if evs:
        per_step.extend(evs[i].elapsed_time(evs[i + 1]) for i in range(steps))
    kt = {}
    if timed_kernels:
        import paper_1711_02242_amd._lib as L
        for g in L.KERNEL_GROUPS:
            ms, n = gs.kernel_time(g)
            kt[g] = (ms, n)
        gs.kernel_timing(False)
    e = gs.energy(wk)
    return gs, wk, (t1 - t0), kt, e


def estimator_report(gs, wk, e):
    """The mixed estimate at the end of the timed steps, the population's E_T and cap centre
    (growth phase), and how often the rare-event bounds bound over the timed steps."""
    e_t, e_bar = gs.growth(wk)
    c = gs.bound_counts()
    live = max(c[3], 1)
    return {"e_mix": e[0] / e[2], "e_trial": e_t, "cap_centre": e_bar,
            "cap_half_width": math.sqrt(gs.params.el_cap_C / gs.dtau),
            "capped_local_energy_fraction": c[0] / live, "capped_weight_fraction": c[1] / live,
            "capped_force_bias_components": c[2], "walker_steps_counted": c[3],
            "fp64_guard_fraction": c[4] / live,
            "alive": e[3], "status": e[4]}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(s, args):
    """The oracle as it stands, on a bounded sample of the same workload."""
    import numpy as np

    from oracle import afqmc as A
    from synthetic import comb_uniform, gaussian_fields
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    S = A.setup(s.h0, s.h1, s.L, s.phi_up, s.phi_dn, args.dtau)
    P = A.Params(dtau=args.dtau)
    nw, nsteps = args.cpu_walkers, args.cpu_steps
    wk = A.init_walkers(S, nw)
    t0 = time.perf_counter()
    for k in range(nsteps):
        x = gaussian_fields(args.seed, 0, wk.walker_id, k, s.n_chol)
        A.step(S, P, wk, x, comb_uniform(args.seed, 0, k))
    dt = time.perf_counter() - t0
    out = {"value": nw * nsteps / dt, "unit": "walker-steps/s", "cores": int(cores),
           "kind": "oracle", "cpu_count": os.cpu_count(), "cpu_model": cpu_model(),
           "sample": f"{nw} walkers x {nsteps} steps of the same workload (NumPy FP64, "
                     f"{dt:.1f} s)"}
    # the same oracle on one thread, on a smaller sample
    try:
        from threadpoolctl import threadpool_limits
        nw1 = max(1, min(4, nw))
        w1 = A.init_walkers(S, nw1)
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            x = gaussian_fields(args.seed, 0, w1.walker_id, 0, s.n_chol)
            A.step(S, P, w1, x, comb_uniform(args.seed, 0, 0))
            d1 = time.perf_counter() - t0
        out["one_thread"] = {"value": nw1 / d1, "unit": "walker-steps/s",
                             "sample": f"{nw1} walkers x 1 step ({d1:.1f} s)"}
    except ImportError:
        pass
    return out


def batch_leg(args):
    """Uneven batch: 24 systems (M uniform on 24..160, N = M/4, N_g = 6M, 128-2048 walkers),
    FP32 bulk.  The same systems and walkers are stepped (a) by per-system launches with the
    default tiles, one system after the other on one stream, and (b) by one graph launch per
    step with autotuned tiles.  Returns the comparison (whole-batch walker-steps/s)."""
    import torch

    import paper_1711_02242_amd as afq
    from synthetic import batch_workload, gen_system
    specs = batch_workload(args.batch_systems)
    t0 = time.perf_counter()
    pairs = []
    for sp in specs:
        s = gen_system(sp["M"], sp["N"], sp["n_chol"], seed=sp["seed"])
        gs = afq.System.from_synthetic(s, dtau=0.005, precision="fp32")
        wk = gs.walkers(sp["n_walkers"])
        gs.init(wk)
        pairs.append((gs, wk))
        del s
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    nw_total = sum(sp["n_walkers"] for sp in specs)
    flops = sum(contraction_flops(sp["M"], sp["N"], sp["N"], sp["n_chol"], sp["n_walkers"])
                for sp in specs)
    eprint(f"bench: batch of {len(specs)} systems, {nw_total} walkers, setup {t_setup:.1f} s")

    def per_system(nsteps):
        for _ in range(nsteps):
            for (gs, wk), sp in zip(pairs, specs):
                gs.step(wk, seed=sp["seed"])

    per_system(args.batch_warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per_system(args.batch_steps)
    torch.cuda.synchronize()
    dt_a = time.perf_counter() - t0

    t0 = time.perf_counter()
    b = afq.Batch(pairs, autotune=True)
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t0
    seeds = [sp["seed"] for sp in specs]
    for _ in range(max(args.batch_warmup, 5)):   # captures the graphs of every phase
        b.step(seeds)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batch_steps):
        b.step(seeds)
    torch.cuda.synchronize()
    dt_b = time.perf_counter() - t0
    tiles = {}
    for t in b.tiles:
        tiles[t] = tiles.get(t, 0) + 1
    b.close()
    for gs, _ in pairs:
        gs.close()
    va = nw_total * args.batch_steps / dt_a
    vb = nw_total * args.batch_steps / dt_b
    eprint(f"bench: batch per-system {1e3 * dt_a / args.batch_steps:.2f} ms/step, "
           f"graph+autotune {1e3 * dt_b / args.batch_steps:.2f} ms/step")
    return {"workload": f"{len(specs)} synthetic systems, M uniform on 24..160, N=M/4, "
                        "N_g=6M, 128-2048 walkers (log-uniform), fp32 bulk, dtau=0.005",
            "systems": len(specs), "walkers_total": nw_total,
            "steps": args.batch_steps, "contraction_tflop_per_step": round(flops / 1e12, 3),
            "per_system_launches": {"value": round(va, 1), "unit": "walker-steps/s",
                                    "ms_per_step": round(1e3 * dt_a / args.batch_steps, 3)},
            "graph_autotuned": {"value": round(vb, 1), "unit": "walker-steps/s",
                                "ms_per_step": round(1e3 * dt_b / args.batch_steps, 3),
                                "tiles": tiles, "autotune_s": round(t_tune, 2)},
            "speedup": round(vb / va, 3),
            "useful_contraction_tflops": round(flops / (dt_b / args.batch_steps) / 1e12, 2),
            "setup_s": round(t_setup, 1)}


def serving_leg(args):
    """Serving: the first jobs of a Poisson(4/s) trace (M uniform on 32..200, N=M/4, N_g=6M,
    256-2048 walkers) replayed in real time through the continuous-batching server, FP32 bulk,
    each job run to its target standard error (1 mHa) or its step cap.  Time-to-energy
    percentiles are taken over the jobs that reached the target only; every job's reblocked
    error and the steps it would need at its measured rate of error decrease are reported.
    The serial plain-FP64 figure times every job alone in FP64 over 25 steps (five QR and comb
    cycles), multiplies that step time by the steps the job took, and queues the jobs
    first-come-first-served on the same arrival times."""
    import numpy as np
    import torch

    import paper_1711_02242_amd as afq
    from paper_1711_02242_amd.serve import JobSpec, Server
    from synthetic import gen_system, serving_trace
    trace = serving_trace(args.serve_jobs)

    def job_specs(scale):
        """The trace's jobs with arrival times multiplied by ``scale``."""
        specs = []
        for t in trace:
            make = (lambda t=t: gen_system(t["M"], t["N"], t["n_chol"], seed=t["seed"]))
            specs.append(JobSpec(t["job_id"], make, t["M"], t["N"], t["N"], t["n_chol"],
                                 t["n_walkers"], t["seed"], precision="fp32", dtau=0.005,
                                 target_stderr=args.serve_target, max_steps=args.serve_steps,
                                 discard=min(200, args.serve_steps // 2),
                                 arrival=t["arrival"] * scale))
        return specs

    def serve(specs):
        srv = Server(int(args.serve_budget_gib * (1 << 30)), check_every=50, autotune=True)
        t0 = time.perf_counter()
        res = srv.run(specs, realtime=True)
        makespan = time.perf_counter() - t0
        tte = np.array([r.time_to_energy for r in res])
        ws = sum(r.steps * sp.n_walkers for r, sp in zip(res, specs))
        eprint(f"bench: served {len(res)} jobs in {makespan:.1f} s, max resident "
               f"{srv.max_resident}, time to retirement p50 {np.percentile(tte, 50):.1f} s p99 "
               f"{np.percentile(tte, 99):.1f} s, {sum(reached(r) for r in res)} at the target")
        return res, tte, ws, makespan, srv.max_resident

    def reached(r):
        return bool(r.plateau and r.stderr < args.serve_target)

    def tte_stats(res, tte):
        ok = np.array([reached(r) for r in res])
        out = {"reached_target": int(ok.sum()), "jobs": len(res),
               "p50_time_to_energy_s": None, "p99_time_to_energy_s": None,
               "p50_time_to_retirement_s": round(float(np.percentile(tte, 50)), 2),
               "p99_time_to_retirement_s": round(float(np.percentile(tte, 99)), 2)}
        if ok.any():
            out["p50_time_to_energy_s"] = round(float(np.percentile(tte[ok], 50)), 2)
            out["p99_time_to_energy_s"] = round(float(np.percentile(tte[ok], 99)), 2)
        return out

    specs = job_specs(1.0)
    res, tte, ws, makespan, max_res = serve(specs)
    # serial plain FP64: per-job step time alone, FIFO over the same arrivals
    t_end, serial_tte, fp64_ms = 0.0, [], []
    for r, sp in zip(res, specs):
        s = sp.make_system()
        gs = afq.System.from_synthetic(s, dtau=sp.dtau, precision="fp64")
        wk = gs.walkers(sp.n_walkers)
        gs.init(wk)
        gs.step(wk, seed=sp.seed, job_id=sp.job_id)
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(args.serve_fp64_steps):
            gs.step(wk, seed=sp.seed, job_id=sp.job_id)
        torch.cuda.synchronize()
        per = (time.perf_counter() - a) / args.serve_fp64_steps
        fp64_ms.append(1e3 * per)
        eprint(f"bench: serial FP64 job {len(fp64_ms)}/{len(specs)} (M={sp.M}, "
               f"{sp.n_walkers} walkers): {1e3 * per:.2f} ms/step")
        gs.close()
        del s
        start = max(sp.arrival, t_end)
        t_end = start + per * r.steps
        serial_tte.append(t_end - sp.arrival)
    serial_tte = np.array(serial_tte)
    jobs = []
    for r, sp in zip(res, specs):
        n_est = max(r.steps - sp.discard, 1)
        need = (sp.discard + n_est * (r.stderr / args.serve_target) ** 2
                if np.isfinite(r.stderr) else None)
        jobs.append({"job": r.job_id, "M": sp.M, "walkers": sp.n_walkers, "steps": r.steps,
                     "energy": round(r.energy, 5), "stderr_ha": round(r.stderr, 5),
                     "plateau": bool(r.plateau),
                     "steps_to_target_at_this_rate": None if need is None else int(need)})
    out = {"workload": f"first {len(specs)} jobs of a Poisson(4/s) trace: M uniform on 32..200, "
                       "N=M/4, N_g=6M, 256-2048 walkers, fp32 bulk, dtau=0.005",
           "hbm_budget_gib": args.serve_budget_gib,
           "target_stderr_ha": args.serve_target, "step_cap": args.serve_steps,
           **tte_stats(res, tte),
           "walker_steps_per_s": round(ws / makespan, 1), "makespan_s": round(makespan, 2),
           "max_resident": max_res, "per_job": jobs,
           "serial_fp64": {**tte_stats(res, serial_tte),
                           "walker_steps_per_s": round(ws / float(t_end), 1),
                           "step_ms_per_job": [round(v, 2) for v in fp64_ms],
                           "method": f"each job alone in FP64, its step time measured over "
                                     f"{args.serve_fp64_steps} steps and multiplied by the "
                                     "steps it took in the served run, FIFO on the arrivals"}}
    if args.serve_load > 0:
        # the same jobs arriving at a fraction of the measured capacity: the trace's arrivals
        # (4/s) keep the server saturated, so its jobs per second of makespan is the capacity
        cap = len(res) / makespan
        rate = args.serve_load * cap
        res2, tte2, ws2, mk2, mr2 = serve(job_specs(4.0 / rate))
        out["at_load"] = {"load": args.serve_load, "capacity_jobs_per_s": round(cap, 4),
                          "arrival_rate_jobs_per_s": round(rate, 4), **tte_stats(res2, tte2),
                          "walker_steps_per_s": round(ws2 / mk2, 1), "makespan_s": round(mk2, 2),
                          "max_resident": mr2}
    return out


def el_error(s, args, gs, wk):
    """Per-walker local-energy error of this precision on the current walkers: against the
    GPU FP64 path on every walker, and against the FP64 oracle on a sample."""
    import numpy as np
    import torch

    import paper_1711_02242_amd as afq
    from oracle import afqmc as A
    ref = afq.System.from_synthetic(s, dtau=args.dtau, precision="fp64")
    wr = ref.walkers(wk.n)
    ref.init(wr)
    wr.U.copy_(wk.U)
    wr.weight.copy_(wk.weight)
    gs.measure(wk)
    ref.measure(wr)
    torch.cuda.synchronize()
    alive = (wk.weight > 0).cpu().numpy()
    e_lo = wk.e_loc.cpu().numpy()[alive]
    e_64 = wr.e_loc.cpu().numpy()[alive]
    err_gpu64 = float(np.abs(e_lo - e_64).max())
    U = wk.U.cpu().numpy()
    S = A.setup(s.h0, s.h1, s.L, s.phi_up, s.phi_dn, args.dtau)
    idx = np.nonzero(alive)[0][: args.oracle_sample]
    err_or = 0.0
    e_all = wk.e_loc.cpu().numpy()
    for w in idx:
        Uu = U[w, : s.n_up, :].T
        Ud = U[w, s.n_up:, :].T
        _, _, e, _ = A.measure(S, Uu, Ud)
        err_or = max(err_or, abs(e_all[w] - e))
    ref.close()
    return err_gpu64, float(err_or), int(len(idx))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--walkers", type=int, default=1024)
    ap.add_argument("--dtau", type=float, default=0.005)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the plain-FP64 GPU run and the local-energy error measurement")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-walkers", type=int, default=64)
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--oracle-sample", type=int, default=4)
    ap.add_argument("--no-closed-shell", action="store_true",
                    help="skip the closed-shell one-spin measurement")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the uneven multi-system batch comparison")
    ap.add_argument("--batch-systems", type=int, default=24)
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--batch-warmup", type=int, default=2)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-loop trace")
    ap.add_argument("--serve-jobs", type=int, default=8)
    ap.add_argument("--serve-steps", type=int, default=300, help="step cap per job")
    ap.add_argument("--serve-target", type=float, default=0.001, help="target stderr (Ha)")
    ap.add_argument("--serve-budget-gib", type=float, default=128.0)
    ap.add_argument("--serve-fp64-steps", type=int, default=25)
    ap.add_argument("--serve-load", type=float, default=0.7,
                    help="rerun the jobs arriving at this fraction of the measured capacity "
                         "(0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 256 MiB device copy first (reference for PMC byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU only; the walker-parallel multi-GPU path "
              "is a design (local comb per GPU, all-reduce of the estimator sums), not code. "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from synthetic import config_system
    torch.cuda.set_device(0)
    s = config_system("large")
    if args.copy_calibration:
        n = 64 << 20
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        b = a.clone()
        torch.cuda.synchronize()
        del a, b
    eprint(f"bench: M={s.M} N={s.n_up}+{s.n_dn} G={s.n_chol} walkers={args.walkers} "
           f"precision={args.precision} steps={args.steps} warmup={args.warmup}")

    step_ms = []
    gs, wk, dt, kt, e = run_gpu(s, args, args.precision, args.steps, args.warmup,
                                per_step=step_ms)
    ms_step = 1e3 * dt / args.steps
    value = args.walkers * args.steps / dt
    ms_c, n_c = kt["contract"]
    flops = contraction_flops(s.M, s.n_up, s.n_dn, s.n_chol, args.walkers)
    avg_s = (ms_c / max(n_c, 1)) * 1e-3
    achieved = flops / avg_s / 1e12
    peak = PEAK_TFLOPS[args.precision]
    # attainable rate of the same MFMA instruction family (register-only microbenchmark, run
    # after the timed region): the clock the device holds under MFMA load shows here
    import paper_1711_02242_amd as afq
    att = afq.mfma_peak(args.precision) / (3.0 if args.precision == "bf16x3" else 1.0)
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": recorded_traffic(args.precision),
                "traffic_unit": "bytes/launch",
                "kernel": "local-energy contraction", "avg_launch_ms": round(ms_c / max(n_c, 1), 4),
                "flops_per_launch": flops, "attainable": round(att, 2),
                "frac_attainable": round(achieved / att, 4),
                "mfma_busy_rocprof": recorded_mfma_busy(args.precision),
                "attainable_method": "afqmc_mfma_peak: register-only MFMA chains on every SIMD"}
    kernels_ms = {k: round(v[0] / max(args.steps, 1), 4) for k, v in kt.items()}
    eprint(f"bench: {ms_step:.3f} ms/step, {value:.1f} walker-steps/s; per-step kernel ms {kernels_ms}")
    est = estimator_report(gs, wk, e)
    eprint(f"bench: E_mix = {e[0] / e[2]:.8f}, alive {e[3]}, status {e[4]:#x}, E_T "
           f"{est['e_trial']:.6f}, cap centre {est['cap_centre']:.6f}, capped E_L fraction "
           f"{est['capped_local_energy_fraction']:.4f}")

    out = {"metric": "walker-steps/s at M=128,N=32,Ng=800 (phaseless AFQMC step)",
           "value": round(value, 2), "unit": "walker-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": DTYPE[args.precision], "data": "synthetic",
           "config": {"workload": "synthetic molecule M=128 N_up=N_dn=32 N_g=800, 1024 walkers, "
                                  "dtau=0.005, QR and comb every 5 steps",
                      "M": s.M, "n_up": s.n_up, "n_dn": s.n_dn, "n_chol": s.n_chol,
                      "n_walkers": args.walkers, "precision": args.precision},
           "roofline": roofline, "kernel_ms_per_step": kernels_ms,
           "step_ms": {"median": round(float(np.median(step_ms)), 4),
                       "p90": round(float(np.percentile(step_ms, 90)), 4),
                       "min": round(min(step_ms), 4), "max": round(max(step_ms), 4),
                       "note": "HIP events per step; every 5th step adds the QR and the comb"},
           "e_mix": e[0] / e[2], "estimator": est}

    if args.precision != "fp64" and not args.no_compare:
        err64, err_or, n_or = el_error(s, args, gs, wk)
        out["el_error_ha"] = {"vs_gpu_fp64_all_walkers": err64, "vs_oracle_sample": err_or,
                              "oracle_sample_walkers": n_or}
        gs.close()
        n64 = max(4, args.steps // 4)
        g2, w2, dt2, kt2, e2 = run_gpu(s, args, "fp64", n64, 2, timed_kernels=False)
        v64 = args.walkers * n64 / dt2
        out["fp64_gpu"] = {"value": round(v64, 2), "unit": "walker-steps/s",
                           "ms_per_step": round(1e3 * dt2 / n64, 3),
                           "speedup_vs_fp64": round(value / v64, 3)}
        g2.close()
    else:
        gs.close()

    if args.precision == "fp32" and not args.no_compare:
        # the BF16x3 split-product bulk on the same workload (local-energy error reported)
        g4, w4, dt4, kt4, e4 = run_gpu(s, args, "bf16x3", args.steps, 2)
        ms4, n4 = kt4["contract"]
        ach4 = flops / ((ms4 / max(n4, 1)) * 1e-3) / 1e12
        err4, _, _ = el_error(s, args, g4, w4)
        out["bf16x3"] = {"value": round(args.walkers * args.steps / dt4, 2),
                         "unit": "walker-steps/s", "ms_per_step": round(1e3 * dt4 / args.steps, 3),
                         "contraction_fp32_equivalent_tflops": round(ach4, 2),
                         "contraction_frac_of_bf16_peak_over_3": round(ach4 / PEAK_TFLOPS["bf16x3"], 4),
                         "contraction_frac_of_attainable_bf16_over_3":
                             round(ach4 / (afq.mfma_peak("bf16x3") / 3.0), 4),
                         "el_error_ha_vs_gpu_fp64_all_walkers": err4}
        g4.close()

    if not args.no_closed_shell and not args.no_compare:
        # the same workload on the closed-shell path (U_up = U_dn stored once; identical results)
        g3, w3, dt3, kt3, e3 = run_gpu(s, args, args.precision, args.steps, 2,
                                       timed_kernels=False, closed_shell=True)
        out["closed_shell"] = {"value": round(args.walkers * args.steps / dt3, 2),
                               "unit": "walker-steps/s",
                               "ms_per_step": round(1e3 * dt3 / args.steps, 3),
                               "e_mix": e3[0] / e3[2]}
        g3.close()

    if not args.no_batch:
        out["batch"] = batch_leg(args)

    if not args.no_serve:
        out["serving"] = serving_leg(args)

    if not args.no_cpu:
        cb = cpu_baseline(s, args)
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
