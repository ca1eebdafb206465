"""Statistical gate: equilibrium observables of the GPU checkerboard sampler
(frozen-field dE of Sec. 3.2) against the FP64 oracle's sequential exact-dE
sampler (Sec. 2.2), within 3 combined standard errors.

The oracle numbers are stored in tests/golden/stats_*.json, written by
tests/golden/make_golden_stats.py (which calls only the oracle).  The GPU
runs the same chains (same seeds, same initial states, same burn-in and
sampling) and derives the same statistics: batch means (20 batches) for
|M|, M_par, and the cone angle eta of eq. (17) from per-batch site
accumulators with a jackknife over batches; each side's standard error is
the larger of the combined batch-means error and the spread of its
independent chains.  Chains of the two samplers
differ move by move (different update order), so only the statistics are
compared.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

from paper_1211_6234_amd import ddmc

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
NBATCH = 20
GATED = ("MABS", "MPAR", "ETA")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ddmc.lib()


def gpu_chain_stats(L, M, reps, nsweeps, prec, algo, coset_l=None):
    """coset_l: run the l-coset schedule (Sec. 3.1) instead of the
    checkerboard, from the same initial states and sweep indices."""
    R = len(reps)
    burn = nsweeps // 5
    nsamp = nsweeps - burn
    nsamp -= nsamp % NBATCH
    per = nsamp // NBATCH
    N = L * L
    with ddmc.Plan(L, M, R, prec=prec, algo=algo) as plan:
        dp = ddmc.replica_params_upload(reps)
        s = plan.spins(R)
        ddmc.init_spins(plan, R, dp, s)
        ctr = torch.zeros(R, dtype=torch.int64, device="cuda")

        def sweeps(first, n):
            if coset_l:
                ddmc.metropolis_sweep_coset(plan, R, dp, s, coset_l, ctr, n)
            else:
                ddmc.metropolis_sweep(plan, R, dp, s, first, n)

        sweeps(0, burn)
        eta = torch.zeros((NBATCH, R, N), dtype=torch.float64, device="cuda")
        outs = torch.zeros((nsamp, R, ddmc.NOBS), dtype=torch.float64, device="cuda")
        for k in range(nsamp):
            sweeps(burn + k, 1)
            ddmc.observables(plan, R, dp, s, None, outs[k], eta[k // per])
        torch.cuda.synchronize()
        obs = outs.cpu().numpy()
        acc = eta.cpu().numpy()
    res = []
    for r in range(R):
        c = {}
        for name in ("MABS", "MPAR"):
            x = obs[:, r, ddmc.OBS[name]]
            b = x.reshape(NBATCH, -1).mean(axis=1)
            c[name] = {"mean": float(x.mean()), "se": float(b.std(ddof=1) / math.sqrt(NBATCH))}
        a = acc[:, r, :]

        def eta_of(sums, n):
            return float(np.mean(np.sqrt((2 / math.pi) ** 2 * sums / n)))

        full = eta_of(a.sum(axis=0), nsamp)
        jk = np.array([eta_of(a.sum(axis=0) - a[b], nsamp - per) for b in range(NBATCH)])
        c["ETA"] = {"mean": full, "se": math.sqrt((NBATCH - 1) / NBATCH * np.sum((jk - jk.mean()) ** 2))}
        res.append(c)
    comb = {}
    for name in GATED:
        m = np.array([c[name]["mean"] for c in res])
        se = np.array([c[name]["se"] for c in res])
        comb[name] = {"mean": float(m.mean()), "se": float(math.sqrt(np.sum(se ** 2)) / len(m)),
                      "chain_spread_se": float(m.std(ddof=1) / math.sqrt(len(m))) if len(m) > 1 else None}
    return comb


def _se(d):
    """Larger of the batch-means SE and the spread of independent chains (the
    latter catches autocorrelation longer than a batch)."""
    return max(d["se"], d.get("chain_spread_se") or 0.0)


def _gate(gpu, ref, label):
    report = []
    ok = True
    for name in GATED:
        d = gpu[name]["mean"] - ref[name]["mean"]
        sg, so = _se(gpu[name]), _se(ref[name])
        s = math.sqrt(sg ** 2 + so ** 2)
        report.append("%s %s: gpu %.5f +- %.5f  oracle %.5f +- %.5f  (%.2f sigma)" % (
            label, name, gpu[name]["mean"], sg, ref[name]["mean"], so, d / s))
        ok = ok and abs(d) <= 3 * s
    print("\n".join(report), flush=True)
    assert ok, "\n".join(report)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("algo", ["direct", "fft", "fft_lds"])
def test_equilibrium_L16(prec, algo):
    ref = json.load(open(os.path.join(HERE, "golden", "stats_L16.json")))
    reps = [dict(p) for p in ([ref["params"]] * len(ref["chains"]))]
    for r, c in enumerate(ref["chains"]):
        reps[r]["seed"] = c["seed"]
        reps[r]["replica_id"] = 0
    gpu = gpu_chain_stats(ref["L"], ref["M"], reps, ref["chains"][0]["sweeps"], prec, algo)
    _gate(gpu, ref["combined"], "L16 %s %s" % (algo, prec))


@pytest.mark.parametrize("prec,algo", [("f64", "fft"), ("f32", "fft"), ("f32", "fft_lds")])
@pytest.mark.parametrize("T", ["T0.5", "T0.8"])
def test_equilibrium_L64(prec, algo, T):
    path = os.path.join(HERE, "golden", "stats_L64.json")
    if not os.path.exists(path):
        pytest.skip("oracle statistics for L = 64 not generated")
    ref = json.load(open(path))[T]
    reps = []
    for c in ref["chains"]:
        p = dict(ref["params"])
        p["seed"] = c["seed"]
        p["replica_id"] = 0
        reps.append(p)
    gpu = gpu_chain_stats(ref["L"], ref["M"], reps, ref["chains"][0]["sweeps"], prec, algo)
    _gate(gpu, ref["combined"], "L64 %s %s %s" % (T, algo, prec))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("l", [8, 4])
def test_equilibrium_L16_coset(prec, l):
    """The l-coset schedule (4 or 16 sites moved at once on the frozen field)
    samples the same equilibrium as the oracle's exact sequential sampler:
    its bias, bounded by eq. (10), is below the statistical error here."""
    ref = json.load(open(os.path.join(HERE, "golden", "stats_L16.json")))
    reps = [dict(p) for p in ([ref["params"]] * len(ref["chains"]))]
    for r, c in enumerate(ref["chains"]):
        reps[r]["seed"] = c["seed"]
        reps[r]["replica_id"] = 0
    gpu = gpu_chain_stats(ref["L"], ref["M"], reps, ref["chains"][0]["sweeps"], prec, "fft", coset_l=l)
    _gate(gpu, ref["combined"], "L16 coset l=%d %s" % (l, prec))


@pytest.mark.parametrize("T", ["T0.5", "T0.8"])
def test_equilibrium_L64_coset(T):
    """The paper's own schedule at its size, L = 64, l = 32 (eq. (10) bound
    1.4e-4 C_D), FP32, against the oracle's exact sequential sampler."""
    path = os.path.join(HERE, "golden", "stats_L64.json")
    if not os.path.exists(path):
        pytest.skip("oracle statistics for L = 64 not generated")
    ref = json.load(open(path))[T]
    reps = []
    for c in ref["chains"]:
        p = dict(ref["params"])
        p["seed"] = c["seed"]
        p["replica_id"] = 0
        reps.append(p)
    gpu = gpu_chain_stats(ref["L"], ref["M"], reps, ref["chains"][0]["sweeps"], "f32", "fft", coset_l=32)
    _gate(gpu, ref["combined"], "L64 coset l=32 %s" % T)
