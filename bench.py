"""Benchmark of the hot path on one MI355X: spin-update attempts per second.

Workload: the batched temperature ladder, L = 128 (N = 16384 spins), R = 32
replicas with T linearly spaced over [0.3, 1.2], g = 0.15, J = 1, K2 = 2,
K4 = 0, images |a|, |b| <= 8, FP32.  One step is one pass of the whole hot
path over the batch: a checkerboard sweep (two half-sweeps, each = local
field of the current state + colour update) followed by one observables
sample (energies, magnetizations, wall counts, cone-angle accumulators),
run as metropolis_sample calls of G steps captured in a HIP graph (the sweep
index lives on the device, so every replay continues the chains).  The kernel
W is built once per lattice size, before the timed region.  An attempt is
one Metropolis proposal at one site; a step is R * N attempts.

Printed (rank 0, one JSON line): the metric, whole-job attempts/s, the
plain form (FP32 direct field, one replica per call) beside it, the
roofline of the dominant kernel measured with HIP events on the stream it
runs on, p50/p99 request latency of a served Poisson mix, and the FP64 CPU
oracle timed on the host on a bounded sample.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spin-update attempts/sec at L=128×32 replicas vs plain; p50/p99 req latency"
HBM_PEAK_GBS = 8000.0
# FP32 VALU peak without packed-FP32 instructions: 256 CU x 4 SIMD x 16 lanes
# x 2 flop (FMA) x 2.4 GHz
FP32_VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--algo", default="auto", choices=["auto", "direct", "fft"])
    ap.add_argument("--plain-steps", type=int, default=10)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-coset", action="store_true")
    ap.add_argument("--no-batch-scaling", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the timed step and its kernel timing (for profiler runs)")
    ap.add_argument("--cpu-sweeps", type=int, default=3)
    ap.add_argument("--prof-steps", type=int, default=50)
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-warmup", type=int, default=50)
    ap.add_argument("--graph-steps", type=int, default=50,
                    help="steps per metropolis_sample call, captured in a HIP graph (0: eager one-step calls)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def host_cpu():
    """Host CPU model and core counts (the oracle's threads are reported apart)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count() or 1
    return {"model": model, "nproc": os.cpu_count(), "affinity": aff}


def cpu_baseline(cfg, sweeps):
    """FP64 oracle, sequential single-spin Metropolis with the exact dE, one
    replica per host thread (at most 16, the host share of one GPU); times
    `sweeps` sweeps after the exact initial field (the oracle's O(N^2) field
    and W build are outside the timing)."""
    import oracle
    L, M = cfg["L"], cfg["M"]
    host = host_cpu()
    threads = max(1, min(16, host["affinity"], len(cfg["replicas"])))
    W = oracle.lattice_sum_kernel(L, M)
    reps = cfg["replicas"][:threads]
    states = []
    for p in reps:
        s = oracle.init_spins(L, p["seed"], p["replica_id"])
        states.append(s)

    def prep(k):
        return oracle.field(L, W, states[k])

    with cf.ThreadPoolExecutor(threads) as ex:
        fields = list(ex.map(prep, range(threads)))

    def run(k):
        p = reps[k]
        op = oracle.params(p["T"], p["J"], p["K2"], p["K4"], p["g"], p["seed"], p["replica_id"])
        return oracle.sweep_sequential(L, W, op, states[k], fields[k], 1, sweeps)

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(run, range(threads)))
    dt = time.perf_counter() - t0
    attempts = threads * sweeps * L * L
    return {"value": attempts / dt, "unit": "attempts/s", "cores": threads, "kind": "oracle",
            "per_core": attempts / dt / threads, "host_cpu": host["model"], "host_nproc": host["nproc"],
            "host_affinity_cpus": host["affinity"],
            "sample": "%d replicas of the workload (one per thread) x %d sequential exact-dE sweeps, "
                      "L=%d, FP64; %.2f s wall, %.1f thread-s" % (threads, sweeps, L, dt, dt * threads)}


TRAFFIC_SOURCES = ("k_fft.hip", "fft_reg.hpp", "obs_common.hpp", "device_common.hpp")


def kernel_source_hash():
    """sha256 of the sources the FFT-path kernels are compiled from (a
    measured traffic figure applies only to the sources it was taken on)."""
    import hashlib
    h = hashlib.sha256()
    files = [os.path.join(ROOT, "paper_1211_6234_amd", "csrc", f) for f in TRAFFIC_SOURCES]
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, L, R):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (rocprofv3 FETCH_SIZE and WRITE_SIZE, scaled by a plain copy), or None
    when there is none for this workload or the kernels changed since."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_L%d_R%d.txt" % (kernel, L, R))
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def served_mix(n, warm):
    """Poisson stream (50 requests/s) of simulations with L in {32, 48, 64, 96,
    128}, random couplings and 2000 sweeps each, served with continuous
    batching; latency = completion - arrival on the host clock."""
    from paper_1211_6234_amd import serve, workloads
    reqs = [serve.Request(i, q["L"], q["params"], q["sweeps"], q["arrival"])
            for i, q in enumerate(workloads.served_mix(n + warm, arrival_seed=0))]
    srv = serve.Server(hbm_budget_bytes=16 << 30, M=8, prec="f32", slots_per_size=64, chunk_sweeps=200,
                       autotune=True)
    done = srv.run(reqs, realtime=True)
    rep = serve.latency_report(done, srv.wall, srv.attempts, warmup=warm)
    rep["workload"] = "Poisson 50 req/s, L in {32,48,64,96,128}, 2000 sweeps each, FP32; %d warm-up requests" % warm
    rep["hbm_budget_bytes"] = srv.budget
    rep["peak_pool_bytes"] = srv.peak_in_use
    rep["sweep_form"] = {str(L): f for L, f in sorted(srv.forms.items())}
    from paper_1211_6234_amd import tune
    rep["tuned_ms_per_sweep"] = {"L%d_R%d" % (k[0], k[1]): v["ms_per_sweep"] for k, v in tune.report().items()}
    srv.close()
    return rep


def main():
    args = parse()
    if args.headline_only:
        args.no_plain = args.no_cpu = args.no_coset = args.no_batch_scaling = args.no_large = True
        args.serve_requests = 0
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(replicas shard across GPUs with no communication)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1211_6234_amd import ddmc, workloads

    torch.cuda.set_device(0)
    cfg = workloads.ladder_l128(32, 0.0)
    L, M, R = cfg["L"], cfg["M"], len(cfg["replicas"])
    N = L * L
    stream = torch.cuda.current_stream()

    plan = ddmc.Plan(L, M, R, prec="f32", algo=args.algo)
    dp = ddmc.replica_params_upload(cfg["replicas"])
    s = plan.spins(R)
    ddmc.init_spins(plan, R, dp, s)
    G = max(1, min(args.graph_steps, args.steps)) if args.graph_steps > 0 else 1
    obs = torch.zeros((G, R, ddmc.NOBS), dtype=torch.float64, device="cuda")   # one sample per step
    eta = torch.zeros((R, N), dtype=torch.float64, device="cuda")
    acc = torch.zeros(R, dtype=torch.int64, device="cuda")
    counter = torch.zeros(R, dtype=torch.int64, device="cuda")   # device sweep index per replica

    def steps(st, n):
        """n steps in one call: n sweeps, each followed by an observables sample."""
        ddmc.metropolis_sample(plan, R, dp, s, counter, n, obs[:n], eta, acc, st)

    def run(n, st):
        for _ in range(n // G):
            steps(st, G)
        if n % G:
            steps(st, n % G)

    run(args.warmup, stream)
    torch.cuda.synchronize()
    graph = None
    if args.graph_steps > 0:
        # G whole steps captured once in a HIP graph; each replay advances the chains
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            steps(torch.cuda.current_stream(), G)
        torch.cuda.synchronize()
        counter.zero_()
        acc.zero_()
        eta.zero_()
        ddmc.init_spins(plan, R, dp, s, stream)
        run(args.warmup, stream)
        torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    if graph is not None:
        for _ in range(args.steps // G):
            graph.replay()
        if args.steps % G:
            steps(stream, args.steps % G)
    else:
        run(args.steps, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ms_step = ms / args.steps
    value = R * N / (ms_step * 1e-3)
    sweeps_done = args.warmup + args.steps
    acc_rate = float(acc.sum().item()) / (R * N * sweeps_done)
    last_obs = obs[(args.steps - 1) % G].cpu().numpy()

    # ---- per-kernel times: the same calls again with the plan's event profiler
    # on (HIP events recorded on the stream of every instrumented launch)
    # (whole calls of G steps, so that each call's first and last launches are
    # amortized as in the timed graph)
    prof_steps = G * max(1, args.prof_steps // G)
    plan.profile(True)
    run(prof_steps, stream)
    kern = plan.profile_read()
    plan.profile(False)
    es = 4
    spin_bytes = R * 3 * N * es                     # one copy of the spins (= one spectrum)
    eta_bytes = 2 * R * N * 8                       # read + write of the FP64 cone-angle sums
    algo_bytes = {
        "fft_rows_sweep": 3.5 * spin_bytes,         # read h^ and s, write S^, write the colour's spins
        "fft_rows_sample": 3.5 * spin_bytes + eta_bytes,   # the same + read and write the eta sums;
                                                    # the observables use the spins and field on chip
        "fft_columns": 2.0 * spin_bytes,            # read S^, write h^
        "fft_rows": 2.0 * spin_bytes,               # read s, write S^
        "update": 4.0 * R * (N // 2) * 3 * es,      # own spin, neighbours, field, write
    }
    # Each profiled launch is bracketed by its own event pair, which adds the
    # dispatch and completion latency of an eager launch to the interval.  The
    # per-launch excess is measured here as the eager bracketed time of a step
    # minus the graph-timed step, spread over the launches of a step, and taken
    # off every launch: what remains is the kernel's duration inside the graph.
    total_ms = sum(v[0] for v in kern.values())
    n_launch = sum(v[1] for v in kern.values())
    bracket_ms = 0.0
    if n_launch > 0:
        bracket_ms = max(0.0, (total_ms / prof_steps - ms_step) / (n_launch / prof_steps))
    kernels = {}
    for name, (tot, n) in kern.items():
        if n == 0:
            continue
        avg = tot / n - bracket_ms
        rec_k = {"launches": n, "avg_ms": avg, "bracketed_avg_ms": tot / n, "share": tot / max(1e-12, total_ms)}
        if name in algo_bytes:
            rec_k["gbs"] = algo_bytes[name] / (avg * 1e-3) / 1e9
        if name == "direct_field":
            rec_k["tflops"] = 10.0 * R * (N // 2) * N / (avg * 1e-3) / 1e12
        kernels[name] = rec_k
    roofline = None
    if kernels:
        dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches"])
        d = kernels[dom]
        if dom == "direct_field":
            roofline = {"bound": "alu", "kernel": dom, "achieved": d["tflops"], "peak": FP32_VALU_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": d["tflops"] / FP32_VALU_PEAK_TFLOPS, "traffic": None,
                        "avg_launch_ms": d["avg_ms"]}
        else:
            roofline = {"bound": "hbm", "kernel": dom, "achieved": d["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": d["gbs"] / HBM_PEAK_GBS, "traffic": measured_traffic(dom, L, R),
                        "avg_launch_ms": d["avg_ms"], "event_bracket_overhead_ms": bracket_ms,
                        "algorithmic_bytes_per_launch": algo_bytes[dom]}
    # the whole step against HBM: algorithmic bytes of every launch of a step
    step_roofline = None
    if plan.algo == "fft":
        step_bytes = 2 * algo_bytes["fft_columns"] + algo_bytes["fft_rows_sweep"] + algo_bytes["fft_rows_sample"]
        step_roofline = {"bound": "hbm", "bytes_per_step": step_bytes,
                         "achieved": step_bytes / (ms_step * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS}

    # ---- the same chains without the observables (sweeps only), graph-captured
    sweep_only = None
    if plan.algo == "fft" and args.graph_steps > 0:
        s2 = s.clone()
        ctr2 = counter.clone()
        ddmc.metropolis_sweep_dev(plan, R, dp, s2, ctr2, G, None, stream)
        torch.cuda.synchronize()
        g2 = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g2):
            ddmc.metropolis_sweep_dev(plan, R, dp, s2, ctr2, G, None, torch.cuda.current_stream())
        torch.cuda.synchronize()
        q0, q1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = max(1, args.steps // G)
        q0.record(stream)
        for _ in range(reps):
            g2.replay()
        q1.record(stream)
        torch.cuda.synchronize()
        sms = q0.elapsed_time(q1) / (reps * G)
        sweep_only = {"value": R * N / (sms * 1e-3), "unit": "attempts/s", "ms_per_sweep": sms,
                      "form": "metropolis_sweep_dev, %d sweeps per graph, no observables" % G}

    # ---- plain form: FP32 direct field, one replica per call, no batching
    plain = None
    if not args.no_plain:
        pplan = ddmc.Plan(L, M, 1, prec="f32", algo="direct", W64=plan.W64)
        dps = [ddmc.replica_params_upload([p]) for p in cfg["replicas"]]
        ss = [pplan.spins(1) for _ in range(R)]
        outs = [torch.zeros((1, 1, ddmc.NOBS), dtype=torch.float64, device="cuda") for _ in range(R)]
        etas = [torch.zeros((1, N), dtype=torch.float64, device="cuda") for _ in range(R)]
        ctrs = [torch.zeros(1, dtype=torch.int64, device="cuda") for _ in range(R)]
        for r in range(R):
            ddmc.init_spins(pplan, 1, dps[r], ss[r])

        def plain_step(k):
            # the same step (sweep, full field, observables with energies), one replica per call
            for r in range(R):
                ddmc.metropolis_sample(pplan, 1, dps[r], ss[r], ctrs[r], 1, outs[r], etas[r], None, stream)

        plain_step(0)
        torch.cuda.synchronize()
        p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        p0.record(stream)
        for k in range(args.plain_steps):
            plain_step(1 + k)
        p1.record(stream)
        torch.cuda.synchronize()
        pms = p0.elapsed_time(p1) / args.plain_steps
        pval = R * N / (pms * 1e-3)
        plain = {"value": pval, "unit": "attempts/s", "ms_per_step": pms,
                 "form": "FP32 direct field, one replica per call, no graph", "speedup": value / pval}
        pplan.close()
        # the plain FP32 FFT sweep: the same step, one replica per call, eager
        fplan = ddmc.Plan(L, M, 1, prec="f32", algo="fft", W64=plan.W64)
        for r in range(R):
            ddmc.init_spins(fplan, 1, dps[r], ss[r])
            ctrs[r].zero_()

        def fft_step():
            for r in range(R):
                ddmc.metropolis_sample(fplan, 1, dps[r], ss[r], ctrs[r], 1, outs[r], etas[r], None, stream)

        fft_step()
        torch.cuda.synchronize()
        f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        f0.record(stream)
        for k in range(args.plain_steps):
            fft_step()
        f1.record(stream)
        torch.cuda.synchronize()
        fms = f0.elapsed_time(f1) / args.plain_steps
        fval = R * N / (fms * 1e-3)
        plain["fft"] = {"value": fval, "unit": "attempts/s", "ms_per_step": fms,
                        "form": "FP32 FFT field, one replica per call, no graph", "speedup": value / fval}
        fplan.close()

    # ---- the ladder with replica exchange: rounds of 10 sampled sweeps then
    # an exchange attempt between neighbours (parities alternating), graph-captured
    tempering = None
    if plan.algo == "fft" and args.graph_steps > 0 and not args.headline_only:
        sp, cp = s.clone(), counter.clone()
        op = torch.zeros((10, R, ddmc.NOBS), dtype=torch.float64, device="cuda")
        swp = torch.zeros(R, dtype=torch.int64, device="cuda")

        def pt_rounds(st):
            for parity in (0, 1):
                ddmc.metropolis_sample(plan, R, dp, sp, cp, 10, op, None, None, st)
                ddmc.parallel_tempering_swap(plan, R, dp, sp, op[9], cp, parity, swp, st)

        pt_rounds(stream)
        torch.cuda.synchronize()
        g3 = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g3):
            pt_rounds(torch.cuda.current_stream())
        torch.cuda.synchronize()
        swp.zero_()
        reps3 = max(1, args.steps // 20)
        t0e, t1e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0e.record(stream)
        for _ in range(reps3):
            g3.replay()
        t1e.record(stream)
        torch.cuda.synchronize()
        pms = t0e.elapsed_time(t1e) / (reps3 * 20)
        rate = (swp.cpu().numpy()[:R - 1] / float(reps3)).tolist()    # one attempt per pair per replay
        tempering = {"value": R * N / (pms * 1e-3), "unit": "attempts/s", "ms_per_sweep": pms,
                     "form": "metropolis_sample 10 sweeps + parallel_tempering_swap, parities alternating",
                     "swap_acceptance_per_pair": rate}
        # the same rounds on a ladder whose neighbours exchange (L = 32, dT ~ 0.02)
        w32 = workloads.ladder_l32_pt(32)
        R32, L32 = len(w32["replicas"]), w32["L"]
        with ddmc.Plan(L32, w32["M"], R32, prec="f32", algo="fft") as p32:
            dp32 = ddmc.replica_params_upload(w32["replicas"])
            s32 = p32.spins(R32)
            ddmc.init_spins(p32, R32, dp32, s32)
            c32 = torch.zeros(R32, dtype=torch.int64, device="cuda")
            o32 = torch.zeros((10, R32, ddmc.NOBS), dtype=torch.float64, device="cuda")
            sw32 = torch.zeros(R32, dtype=torch.int64, device="cuda")

            def pt32(st):
                for parity in (0, 1):
                    ddmc.metropolis_sample(p32, R32, dp32, s32, c32, 10, o32, None, None, st)
                    ddmc.parallel_tempering_swap(p32, R32, dp32, s32, o32[9], c32, parity, sw32, st)

            for _ in range(50):          # 1000 sweeps to leave the uniform start
                pt32(stream)
            torch.cuda.synchronize()
            g4 = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g4):
                pt32(torch.cuda.current_stream())
            torch.cuda.synchronize()
            sw32.zero_()
            reps4 = 100
            t0e.record(stream)
            for _ in range(reps4):
                g4.replay()
            t1e.record(stream)
            torch.cuda.synchronize()
            pms4 = t0e.elapsed_time(t1e) / (reps4 * 20)
            acc4 = sw32.cpu().numpy()[:R32 - 1] / float(reps4)
            del g4
        tempering["exchanging_ladder"] = {
            "workload": w32["name"], "L": L32, "replicas": R32, "T": [0.6, 1.2],
            "ms_per_sweep": pms4, "value": R32 * L32 * L32 / (pms4 * 1e-3), "unit": "attempts/s",
            "swap_acceptance_mean": float(acc4.mean()), "swap_acceptance_min": float(acc4.min()),
            "swap_acceptance_per_pair": acc4.tolist()}

    # ---- the paper's own l-coset schedule (Sec. 3.1) on the same ladder, for
    # comparison: l = 2 at L = 128, and the paper's L = 64, l = 32 case
    coset = None
    if not args.no_coset:
        coset = []
        for (Lc, lc, nsw) in ((128, 2, 10), (64, 32, 4)):
            reps_c = cfg["replicas"]
            with ddmc.Plan(Lc, M, R, prec="f32", algo="auto") as pc:
                dpc = ddmc.replica_params_upload(reps_c)
                sc = pc.spins(R)
                ddmc.init_spins(pc, R, dpc, sc)
                cc = torch.zeros(R, dtype=torch.int64, device="cuda")
                ddmc.metropolis_sweep_coset(pc, R, dpc, sc, lc, cc, 1, None, stream)
                torch.cuda.synchronize()
                c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                c0.record(stream)
                ddmc.metropolis_sweep_coset(pc, R, dpc, sc, lc, cc, nsw, None, stream)
                c1.record(stream)
                torch.cuda.synchronize()
                cms = c0.elapsed_time(c1) / nsw
                eps = ddmc.coset_error_bound(Lc, lc)
                coset.append({"L": Lc, "l": lc, "replicas": R, "value": R * Lc * Lc / (cms * 1e-3),
                              "unit": "attempts/s", "ms_per_sweep": cms,
                              "eq10_bound_CD": eps})

    # ---- precision: the FP32 field of the benchmark's state against the FP64
    # field of the same state (the FP64 path is the one checked against the
    # oracle to 1e-12), and the rate of the same step computed in FP64
    precision = None
    if plan.algo == "fft" and args.graph_steps > 0 and not args.headline_only:
        with ddmc.Plan(L, M, R, prec="f64", algo="fft", W64=plan.W64) as p64:
            s64 = torch.empty((R, 3, L, L), dtype=torch.float64, device="cuda")
            ddmc.spins_convert(R, L, s, s64, stream)
            h64, h32 = p64.spins(R), plan.spins(R)
            ddmc.local_field(p64, R, s64, h64, -1, stream)
            ddmc.local_field(plan, R, s, h32, -1, stream)
            torch.cuda.synchronize()
            d = (h32.double() - h64).abs().amax(dim=(2, 3))
            ref = h64.abs().amax(dim=(2, 3)).clamp_min(1e-300)
            field_err = float((d / ref).max())
            o64 = torch.zeros((G, R, ddmc.NOBS), dtype=torch.float64, device="cuda")
            e64 = torch.zeros((R, N), dtype=torch.float64, device="cuda")
            k64 = counter.clone()
            ddmc.metropolis_sample(p64, R, dp, s64, k64, G, o64, e64, None, stream)
            torch.cuda.synchronize()
            g64 = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g64):
                ddmc.metropolis_sample(p64, R, dp, s64, k64, G, o64, e64, None, torch.cuda.current_stream())
            g64.replay()
            torch.cuda.synchronize()
            q0, q1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            nrep = max(1, (args.steps // G) // 2)
            q0.record(stream)
            for _ in range(nrep):
                g64.replay()
            q1.record(stream)
            torch.cuda.synchronize()
            ms64 = q0.elapsed_time(q1) / (nrep * G)
            del g64
        precision = {"fp32_field_rel_err_vs_fp64": field_err,
                     "norm": "max over replicas and components of |h32 - h64|_inf / |h64|_inf",
                     "fp64_step": {"value": R * N / (ms64 * 1e-3), "unit": "attempts/s", "ms_per_step": ms64}}

    # ---- the same step on larger ladders of the same recipe (more replicas per
    # launch): how the launch and latency floor of the four launches amortizes
    batch_scaling = None
    if plan.algo == "fft" and args.graph_steps > 0 and not args.no_batch_scaling:
        batch_scaling = []
        for Rb in (64, 128, 256):
            cb = workloads.ladder_l128(Rb, 0.0)
            with ddmc.Plan(L, M, Rb, prec="f32", algo="fft") as pb:
                dpb = ddmc.replica_params_upload(cb["replicas"])
                sb = pb.spins(Rb)
                ddmc.init_spins(pb, Rb, dpb, sb)
                ob = torch.zeros((G, Rb, ddmc.NOBS), dtype=torch.float64, device="cuda")
                eb = torch.zeros((Rb, N), dtype=torch.float64, device="cuda")
                ab = torch.zeros(Rb, dtype=torch.int64, device="cuda")
                kb = torch.zeros(Rb, dtype=torch.int64, device="cuda")
                ddmc.metropolis_sample(pb, Rb, dpb, sb, kb, G, ob, eb, ab, stream)
                torch.cuda.synchronize()
                gb = torch.cuda.CUDAGraph()
                with torch.cuda.graph(gb):
                    ddmc.metropolis_sample(pb, Rb, dpb, sb, kb, G, ob, eb, ab, torch.cuda.current_stream())
                gb.replay()
                torch.cuda.synchronize()
                b0, b1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                nrep = max(1, (args.steps // G) // 2)
                b0.record(stream)
                for _ in range(nrep):
                    gb.replay()
                b1.record(stream)
                torch.cuda.synchronize()
                bms = b0.elapsed_time(b1) / (nrep * G)
                bbytes = step_bytes * Rb / R if step_bytes else None
                batch_scaling.append({"replicas": Rb, "value": Rb * N / (bms * 1e-3), "unit": "attempts/s",
                                      "ms_per_step": bms,
                                      "step_hbm_frac": (bbytes / (bms * 1e-3) / 1e9 / HBM_PEAK_GBS) if bbytes else None})
                del gb

    # ---- the ladder's other anisotropy batches (K4 = -1 and +1), the same
    # graph-captured step
    ladder_k4 = None
    if plan.algo == "fft" and args.graph_steps > 0 and not args.headline_only:
        ladder_k4 = []
        for K4 in (-1.0, 1.0):
            ck = workloads.ladder_l128(R, K4)
            dpk = ddmc.replica_params_upload(ck["replicas"])
            sk = plan.spins(R)
            ddmc.init_spins(plan, R, dpk, sk)
            kk = torch.zeros(R, dtype=torch.int64, device="cuda")
            ok_ = torch.zeros((G, R, ddmc.NOBS), dtype=torch.float64, device="cuda")
            ek = torch.zeros((R, N), dtype=torch.float64, device="cuda")
            ak = torch.zeros(R, dtype=torch.int64, device="cuda")
            ddmc.metropolis_sample(plan, R, dpk, sk, kk, G, ok_, ek, ak, stream)
            torch.cuda.synchronize()
            gk = torch.cuda.CUDAGraph()
            with torch.cuda.graph(gk):
                ddmc.metropolis_sample(plan, R, dpk, sk, kk, G, ok_, ek, ak, torch.cuda.current_stream())
            gk.replay()
            torch.cuda.synchronize()
            k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            nrep = max(1, args.steps // G)
            k0.record(stream)
            for _ in range(nrep):
                gk.replay()
            k1.record(stream)
            torch.cuda.synchronize()
            kms = k0.elapsed_time(k1) / (nrep * G)
            ladder_k4.append({"workload": ck["name"], "K4": K4, "value": R * N / (kms * 1e-3), "unit": "attempts/s",
                              "ms_per_step": kms,
                              "acceptance": float(ak.sum().item()) / (R * N * G * (nrep + 2))})
            del gk

    # ---- small lattices (the served sizes): the sweep with each replica in
    # one workgroup for the whole call against the four-launch FFT sweep,
    # 32 replicas of the ladder recipe, graph-captured calls of G sweeps; and
    # the sampled step (metropolis_sample) in both forms
    small = None
    if args.graph_steps > 0 and not args.headline_only:
        small = []
        # 32 replicas (the benchmark's batch) and 256 (one replica per CU for
        # the one-workgroup form)
        for Rs in (R, 256):
            reps_s = cfg["replicas"] if Rs == R else workloads.ladder_l128(Rs)["replicas"]
            for Ls in (32, 48, 64):
                rec_s = {"L": Ls, "replicas": Rs}
                for algo in ("fft", "fft_lds"):
                    with ddmc.Plan(Ls, M, Rs, prec="f32", algo=algo) as ps:
                        dps = ddmc.replica_params_upload(reps_s)
                        ss = ps.spins(Rs)
                        ddmc.init_spins(ps, Rs, dps, ss)
                        ks = torch.zeros(Rs, dtype=torch.int64, device="cuda")
                        ddmc.metropolis_sweep_dev(ps, Rs, dps, ss, ks, G, None, stream)
                        torch.cuda.synchronize()
                        gs = torch.cuda.CUDAGraph()
                        with torch.cuda.graph(gs):
                            ddmc.metropolis_sweep_dev(ps, Rs, dps, ss, ks, G, None, torch.cuda.current_stream())
                        gs.replay()
                        torch.cuda.synchronize()
                        s0e, s1e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                        nrep = max(1, args.steps // G)
                        s0e.record(stream)
                        for _ in range(nrep):
                            gs.replay()
                        s1e.record(stream)
                        torch.cuda.synchronize()
                        sms = s0e.elapsed_time(s1e) / (nrep * G)
                        rec_s[algo] = {"ms_per_sweep": sms, "value": Rs * Ls * Ls / (sms * 1e-3), "unit": "attempts/s"}
                        del gs
                        # the sampled step (sweep + observables sample, as the
                        # headline step) in the same form
                        os_ = torch.zeros((G, Rs, ddmc.NOBS), dtype=torch.float64, device="cuda")
                        es_ = torch.zeros((Rs, Ls * Ls), dtype=torch.float64, device="cuda")
                        gq = torch.cuda.CUDAGraph()
                        with torch.cuda.graph(gq):
                            ddmc.metropolis_sample(ps, Rs, dps, ss, ks, G, os_, es_, None, torch.cuda.current_stream())
                        gq.replay()
                        torch.cuda.synchronize()
                        q0e, q1e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                        q0e.record(stream)
                        for _ in range(nrep):
                            gq.replay()
                        q1e.record(stream)
                        torch.cuda.synchronize()
                        qms = q0e.elapsed_time(q1e) / (nrep * G)
                        rec_s[algo]["sampled_ms_per_step"] = qms
                        del gq
                small.append(rec_s)

    # ---- the large-lattice workload (L = 256, 64 replicas, FP32 FFT field):
    # the sampled step, and every 100 sweeps a full-energy resync of the state
    # in FP64 (spins converted, FP64 field, FP64 observables) compared with
    # the FP32 path's own energy of the same state
    large = None
    if plan.algo == "fft" and args.graph_steps > 0 and not args.no_large:
        cl = workloads.large_l256(64)
        Ll, Rl = cl["L"], len(cl["replicas"])
        Nl = Ll * Ll
        with ddmc.Plan(Ll, cl["M"], Rl, prec="f32", algo="fft") as pl, \
                ddmc.Plan(Ll, cl["M"], Rl, prec="f64", algo="fft", W64=pl.W64) as pl64:
            dpl = ddmc.replica_params_upload(cl["replicas"])
            sl = pl.spins(Rl)
            ddmc.init_spins(pl, Rl, dpl, sl, stream)
            ol = torch.zeros((G, Rl, ddmc.NOBS), dtype=torch.float64, device="cuda")
            kl = torch.zeros(Rl, dtype=torch.int64, device="cuda")
            ddmc.metropolis_sample(pl, Rl, dpl, sl, kl, G, ol, None, None, stream)
            torch.cuda.synchronize()
            gl = torch.cuda.CUDAGraph()
            with torch.cuda.graph(gl):
                ddmc.metropolis_sample(pl, Rl, dpl, sl, kl, G, ol, None, None, torch.cuda.current_stream())
            gl.replay()
            torch.cuda.synchronize()
            l0, l1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            nrep = max(1, (args.steps // G) // 2)
            l0.record(stream)
            for _ in range(nrep):
                gl.replay()
            l1.record(stream)
            torch.cuda.synchronize()
            lms = l0.elapsed_time(l1) / (nrep * G)
            lbytes = step_bytes * (Rl * Nl) / (R * N) if step_bytes else None
            s64 = torch.empty((Rl, 3, Ll, Ll), dtype=torch.float64, device="cuda")
            h64 = pl64.spins(Rl)
            o64 = torch.zeros((Rl, ddmc.NOBS), dtype=torch.float64, device="cuda")
            per_resync = max(1, 100 // G)
            gaps, rms = [], []
            for _ in range(2):
                for _ in range(per_resync):
                    gl.replay()
                r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                r0.record(stream)
                ddmc.spins_convert(Rl, Ll, sl, s64, stream)
                ddmc.local_field(pl64, Rl, s64, h64, -1, stream)
                ddmc.observables(pl64, Rl, dpl, s64, h64, o64, None, stream)
                r1.record(stream)
                torch.cuda.synchronize()
                rms.append(r0.elapsed_time(r1))
                e32 = ol[G - 1, :, ddmc.OBS["E"]]
                e64 = o64[:, ddmc.OBS["E"]]
                gaps.append(float(((e32 - e64).abs() / e64.abs().clamp_min(1e-300)).max()))
            del gl
        large = {"workload": cl["name"], "L": Ll, "replicas": Rl, "value": Rl * Nl / (lms * 1e-3),
                 "unit": "attempts/s", "ms_per_step": lms,
                 "step_hbm_frac": (lbytes / (lms * 1e-3) / 1e9 / HBM_PEAK_GBS) if lbytes else None,
                 "resync": {"every_sweeps": per_resync * G, "ms": sum(rms) / len(rms),
                            "energy_rel_gap_fp32_vs_fp64": max(gaps),
                            "form": "spins_convert + FP64 local_field + FP64 observables of the same state; "
                                    "gap = max over replicas and resyncs of |E32 - E64| / |E64|"}}

    latency = None
    if args.serve_requests > 0:
        latency = served_mix(args.serve_requests, args.serve_warmup)

    cpu = None if args.no_cpu else cpu_baseline(cfg, args.cpu_sweeps)

    rec = {
        "metric": METRIC, "value": value, "unit": "attempts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": cfg["name"], "L": L, "replicas": R, "M": M, "g": 0.15, "J": 1.0, "K2": 2.0,
                   "K4": 0.0, "T": [0.3, 1.2], "field": plan.algo, "precision": "f32",
                   "step": "1 checkerboard sweep + 1 observables sample",
                   "launch": ("HIP graph of one metropolis_sample call of %d steps" % G) if graph is not None
                   else "eager metropolis_sample calls of %d steps" % G,
                   "acceptance": acc_rate,
                   "last_sample_mean_energy": float(np.mean(last_obs[:, ddmc.OBS["E"]]))},
        "roofline": roofline,
        "step_roofline": step_roofline,
        "sweep_only": sweep_only,
        "kernels": kernels,
        "cpu_baseline": cpu,
        "plain": plain,
        "tempering": tempering,
        "coset": coset,
        "batch_scaling": batch_scaling,
        "ladder_k4": ladder_k4,
        "small_lattices": small,
        "large": large,
        "precision": precision,
        "latency": latency,
    }
    print(json.dumps(rec), flush=True)
    if args.calib_copy_mib > 0:
        # counter calibration: one plain device copy of a known size whose
        # source is no longer in L2 (two larger buffers are written after it)
        n = args.calib_copy_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        evict = [torch.full((n,), 2.0, device="cuda") for _ in range(2)]
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del evict
    plan.close()


if __name__ == "__main__":
    main()
