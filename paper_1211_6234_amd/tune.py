"""Autotuner of the sweep form (host scheduling only).

A checkerboard sweep of a batch of replicas runs in one of two forms, both
in the library's kernels and both sampling the same chains to within the
rounding of the field: the four-launch FFT sweep (row and column blocks
spread over the whole GPU) or, for small lattices, the sweep with each
replica's lattice held in one workgroup for a whole call (DDMC_FIELD_FFT_LDS).
Which is faster depends on the lattice size and the batch: the first is
bound by the latency of its four launches per sweep, the second by one CU's
LDS bandwidth per replica.  `pick` times both forms on the device for a
(L, replicas, precision) shape, graph-captured as they would be served, and
returns the faster; results are cached per shape for the process.  With
sampled=True it times sampled steps (metropolis_sample: a sweep and an
observables sample each) instead, for callers that sample every sweep: the
one-workgroup form then carries the samples in its kernel, at a cost that
grows with the lattice, so the faster form can differ.
"""
from __future__ import annotations

import torch

from . import ddmc, workloads

_cache = {}


def _time_form(L, R, prec, algo, sweeps, reps, sampled=False):
    with ddmc.Plan(L, 4, R, prec=prec, algo=algo) as plan:
        params = [workloads.replica(0.5 + 0.5 * r / max(1, R - 1), 1.0, 1.5, 0.0, 0.15, seed=7 + r, replica_id=r)
                  for r in range(R)]
        dp = ddmc.replica_params_upload(params)
        s = plan.spins(R)
        ddmc.init_spins(plan, R, dp, s)
        ctr = torch.zeros(R, dtype=torch.int64, device="cuda")
        st = torch.cuda.current_stream()
        obs = torch.zeros((sweeps, R, ddmc.NOBS), dtype=torch.float64, device="cuda") if sampled else None

        def call(cs):
            if sampled:
                ddmc.metropolis_sample(plan, R, dp, s, ctr, sweeps, obs, None, None, cs)
            else:
                ddmc.metropolis_sweep_dev(plan, R, dp, s, ctr, sweeps, None, cs)

        call(st)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            call(torch.cuda.current_stream())
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            g.replay()
        e1.record(st)
        torch.cuda.synchronize()
        del g
        return e0.elapsed_time(e1) / (reps * sweeps)


def pick(L, R, prec="f32", sweeps=20, reps=3, sampled=False):
    """'fft_lds' or 'auto' for a batch of R replicas of size L, by measurement
    (ms per sweep, or per sampled step, of each candidate in the record)."""
    key = (int(L), int(R), prec) + (("sampled",) if sampled else ())
    rec = _cache.get(key)
    if rec is not None:
        return rec["form"]
    times = {"auto": _time_form(L, R, prec, "auto", sweeps, reps, sampled)}
    try:
        ddmc.plan_device_bytes(L, R, prec, "fft_lds")
        times["fft_lds"] = _time_form(L, R, prec, "fft_lds", sweeps, reps, sampled)
    except ddmc.DDMCError:
        pass   # no one-workgroup form for this size
    form = min(times, key=times.get)
    _cache[key] = {"form": form, "ms_per_sweep": times}
    return form


def report():
    """Every shape tuned in this process: {(L, R, prec): {form, ms_per_sweep}}."""
    return dict(_cache)
