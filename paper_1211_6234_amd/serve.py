"""Continuous-batching server for independent simulations (host scheduling only).

Each request is one simulation: a lattice size L, replica parameters
(T, J, K2, K4, g, seed) and a number of sweeps.  Requests are admitted as
they arrive while the HBM budget allows; an admitted request's spins live in
a slot of a per-L pool on the device until it completes.  Every scheduling
tick runs a chunk of sweeps for all resident requests of one L in a single
batched ``metropolis_sweep_dev`` call (one launch per chunk for the small
sizes whose replicas each fit in one workgroup; each request keeps its own device
sweep counter, so requests admitted at different times share a launch), with
one HIP stream per lattice size so that the work of different sizes
overlaps on the device.  The chunk call is captured once per (batch bucket,
chunk length) in a HIP graph and replayed, so that a tick costs one graph
launch on the host instead of four kernel launches per sweep; the batch is
the resident requests rounded up to a power of two, the slots beyond them
holding valid idle states.  Each size polls the completion event of its
own chunk and starts the next one as soon as it ends, so sizes do not wait
for each other.  A finished request is sampled with ``observables`` and its
slot is refilled by compaction.

All arithmetic runs in the library's kernels; this module only decides what
to launch.  Because every kernel treats replicas independently and sweep
indices come from the per-request counters, a request's result does not
depend on which other requests shared its launches.
"""
from __future__ import annotations

import collections
import time

import numpy as np
import torch

from . import ddmc


class Request:
    def __init__(self, rid, L, params, sweeps, arrival=0.0):
        self.rid, self.L, self.params, self.sweeps, self.arrival = rid, int(L), dict(params), int(sweeps), arrival
        self.params.setdefault("replica_id", 0)
        self.done_sweeps = 0
        self.t_admit = None
        self.t_done = None
        self.result = None        # observables row (numpy float64 [NOBS]) at completion
        self.accepted = None
        self.state = None         # final spins (host), when the server keeps them

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.arrival


# Sizes whose sweeps run with each replica in one workgroup (DDMC_FIELD_FFT_LDS):
# measured faster there than the four-launch FFT sweep at every batch size
# (FP32 at 32 replicas: 10.8 vs 18.4 us per sweep at L = 32, 17.4 vs 20.1 at
# 48); at L = 64 the four-launch form is faster for the small batches a
# server holds (19.0 vs 22.1 us at 32 replicas) and slower for large ones
# (43.5 vs 24.8 us at 256).
LDS_SIZES = {"f32": (8, 16, 24, 32, 48), "f64": (8, 16, 24, 32)}


def field_algo(L, prec="f32"):
    """The plan form a pool of size L uses."""
    return "fft_lds" if L in LDS_SIZES[prec] else "auto"


def group_bytes(L, cap, prec="f32"):
    """Device bytes a pool of `cap` request slots of size L holds: the plan
    (derived kernel forms and workspace for `cap` replicas, as the library
    reports it) plus the slots' spins, parameter records, sweep counters,
    accept counts and one observables row, and the FP64 kernel W the plan
    is derived from."""
    es = 8 if prec == "f64" else 4
    blk = lambda b: (b + 511) // 512 * 512     # torch's allocator rounds each tensor to 512 bytes
    tensors = (blk(cap * 3 * L * L * es) + blk(cap * ddmc.PARAMS_BYTES) + 2 * blk(cap * 8)
               + blk(ddmc.NOBS * 8) + blk(4 * L * L * 8))
    return ddmc.plan_device_bytes(L, cap, prec, field_algo(L, prec)) + tensors


class _Group:
    """Resident requests of one lattice size: slots 0..n-1 of a device pool
    of `cap` slots, allocated once when the group is created."""

    def __init__(self, L, M, cap, prec, algo):
        self.L, self.cap = L, cap
        self.bytes = group_bytes(L, cap, prec)
        self.stream = torch.cuda.Stream()
        with torch.cuda.stream(self.stream):
            self.plan = ddmc.Plan(L, M, cap, prec=prec, algo=algo, stream=self.stream)
            self.s = self.plan.spins(cap)
            self.params = torch.zeros(cap * ddmc.PARAMS_BYTES, dtype=torch.uint8, device="cuda")
            self.ctr = torch.zeros(cap, dtype=torch.int64, device="cuda")
            self.acc = torch.zeros(cap, dtype=torch.int64, device="cuda")
            self.out = torch.zeros((1, ddmc.NOBS), dtype=torch.float64, device="cuda")
        # every slot holds a valid state from the start, so that idle slots of a
        # rounded-up batch compute on unit spins
        ddmc.init_spins(self.plan, cap, self.params, self.s, stream=self.stream)
        self.reqs = []
        self.graphs = {}   # (batch, chunk) -> captured chunk call
        self.busy = []     # requests of the chunk in flight
        self.done_ev = torch.cuda.Event()

    def close(self):
        self.graphs = {}
        self.stream.synchronize()
        self.plan.close()
        self.s = self.params = self.ctr = self.acc = self.out = None

    def _slot(self, k):
        return (self.s[k:k + 1], self.params[k * ddmc.PARAMS_BYTES:(k + 1) * ddmc.PARAMS_BYTES],
                self.ctr[k:k + 1], self.acc[k:k + 1])

    def admit(self, req):
        """Enqueue the new request's set-up on the group's stream behind any
        chunk in flight; nothing here waits for the device."""
        k = len(self.reqs)
        s, p, c, a = self._slot(k)
        st = self.stream
        ddmc.replica_params_upload([req.params], p, stream=st)
        with torch.cuda.stream(st):
            c.zero_()
            a.zero_()
        ddmc.init_spins(self.plan, 1, p, s, stream=st)
        self.reqs.append(req)

    def _graph(self, nb, chunk):
        g = self.graphs.get((nb, chunk))
        if g is None:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=self.stream):
                ddmc.metropolis_sweep_dev(self.plan, nb, self.params, self.s, self.ctr, chunk, self.acc,
                                          stream=self.stream)
            self.graphs[(nb, chunk)] = g
        return g

    def run_chunk(self, max_chunk):
        """Enqueue one chunk for the resident requests; returns the attempts."""
        n = len(self.reqs)
        chunk = min([max_chunk] + [r.sweeps - r.done_sweeps for r in self.reqs])
        nb = min(self.cap, 1 << (n - 1).bit_length())
        g = self._graph(nb, chunk)
        with torch.cuda.stream(self.stream):
            g.replay()
        self.done_ev.record(self.stream)
        for r in self.reqs:
            r.done_sweeps += chunk
        self.busy = list(self.reqs)
        return n * chunk * self.L * self.L

    def chunk_finished(self):
        """True when no chunk is in flight (polls the device, never blocks)."""
        if self.busy and self.done_ev.query():
            self.busy = []
        return not self.busy

    def retire_finished(self, now, keep_state):
        k = 0
        while k < len(self.reqs):
            r = self.reqs[k]
            if r.done_sweeps < r.sweeps:
                k += 1
                continue
            s, p, c, a = self._slot(k)
            ddmc.observables(self.plan, 1, p, s, None, self.out, None, stream=self.stream)
            self.stream.synchronize()
            r.result = self.out[0].cpu().numpy().copy()
            r.accepted = int(a.item())
            if keep_state:
                r.state = s[0].cpu().numpy().copy()
            r.t_done = now()
            last = len(self.reqs) - 1
            if k != last:   # compaction: move the last resident request into slot k
                s2, p2, c2, a2 = self._slot(last)
                with torch.cuda.stream(self.stream):
                    s.copy_(s2)
                    p.copy_(p2)
                    c.copy_(c2)
                    a.copy_(a2)
                self.reqs[k] = self.reqs[last]
            self.reqs.pop()
            yield r


class Server:
    """Admission by HBM budget, resident state, continuous batching per L.

    The budget bounds the device memory the server allocates: a size's pool
    is created (plan and slot arrays) only when its bytes fit in what the
    budget leaves, with as many slots as fit, up to `slots_per_size`; a
    request is admitted when its size's pool has a free slot.  Pools that
    fall idle are released when another size needs the room."""

    def __init__(self, hbm_budget_bytes=8 << 30, M=8, prec="f32", slots_per_size=64, chunk_sweeps=100,
                 keep_state=False, autotune=False):
        self.budget = int(hbm_budget_bytes)
        self.M, self.prec = M, prec
        self.slots_per_size = slots_per_size
        self.chunk = chunk_sweeps
        self.keep_state = keep_state
        # the sweep form of each size: measured on the device for a batch of up
        # to 8 requests (tune.pick), or the fixed table LDS_SIZES
        self.autotune = autotune
        self.forms = {}
        self.groups = {}
        self.in_use = 0           # bytes of the live pools
        self.peak_in_use = 0
        # device bytes actually held (torch's tensors of the pools plus the
        # library's plans), sampled whenever a pool is created
        self.peak_measured = 0
        self._base_alloc = torch.cuda.memory_allocated()

    def _cap_for(self, L):
        """Most slots (<= slots_per_size) whose pool fits in the budget left."""
        room = self.budget - self.in_use
        lo, hi = 0, self.slots_per_size
        while lo < hi:
            mid = (lo + hi + 1) // 2
            if group_bytes(L, mid, self.prec) <= room:
                lo = mid
            else:
                hi = mid - 1
        return lo

    def _release_idle(self, keep):
        for L in [L for L, g in self.groups.items() if L != keep and not g.reqs and not g.busy]:
            g = self.groups.pop(L)
            self.in_use -= g.bytes
            g.close()

    def _pool_for(self, L):
        """The pool of size L with a free slot, creating it if the budget
        allows; None when the request has to wait."""
        g = self.groups.get(L)
        if g is not None:
            return g if len(g.reqs) < g.cap else None
        cap = self._cap_for(L)
        if cap < 1:
            self._release_idle(keep=L)
            cap = self._cap_for(L)
        if cap < 1:
            return None
        form = self.forms.get(L)
        if form is None:
            if self.autotune:
                from . import tune
                form = tune.pick(L, min(self.slots_per_size, 8), self.prec)
            else:
                form = field_algo(L, self.prec)
            self.forms[L] = form
        g = _Group(L, self.M, cap, self.prec, form)
        self.groups[L] = g
        self.in_use += g.bytes
        self.peak_in_use = max(self.peak_in_use, self.in_use)
        held = torch.cuda.memory_allocated() - self._base_alloc + sum(
            ddmc.plan_device_bytes(q.L, q.cap, self.prec, q.plan.algo) for q in self.groups.values())
        self.peak_measured = max(self.peak_measured, held)
        return g

    def run(self, requests, realtime=True):
        """Serve `requests` (with .arrival seconds); returns them completed, in completion order."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        done = []
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        attempts = 0
        while pending or any(g.reqs for g in self.groups.values()):
            t = now()
            # admission: arrived requests, FIFO, while the budget allows
            while pending and (not realtime or pending[0].arrival <= t):
                r = pending[0]
                if group_bytes(r.L, 1, self.prec) > self.budget:   # can never fit: reject
                    pending.popleft()
                    r.t_done = now()
                    r.result = None
                    done.append(r)
                    continue
                g = self._pool_for(r.L)
                if g is None:
                    break
                pending.popleft()
                r.t_admit = t
                g.admit(r)
            # every size whose previous chunk has finished retires its finished
            # requests and starts its next chunk at once; sizes run independently
            progressed = False
            for g in list(self.groups.values()):
                if not g.chunk_finished():
                    continue
                for r in g.retire_finished(now, self.keep_state):
                    done.append(r)
                    progressed = True
                if g.reqs:
                    attempts += g.run_chunk(self.chunk)
                    progressed = True
            if not progressed:
                busy = any(g.busy for g in self.groups.values())
                if busy:
                    time.sleep(20e-6)
                elif pending:
                    time.sleep(max(0.0, min(0.001, pending[0].arrival - now())))
        self.wall = now()
        self.attempts = attempts
        return done

    def close(self):
        for g in self.groups.values():
            g.close()
        self.groups = {}
        self.in_use = 0


def latency_report(done, wall, attempts, warmup=0):
    lat = np.array([r.latency for r in sorted(done, key=lambda r: r.rid)[warmup:]])
    return {"requests": int(len(lat)), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "attempts_per_s": attempts / wall, "wall_s": wall}
