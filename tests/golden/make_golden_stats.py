"""Write the oracle's equilibrium statistics used by the 3-sigma gates.

Runs only the FP64 CPU oracle (sequential single-spin Metropolis with the
exact dE, Sec. 2.2) on the synthetic workloads, several independent chains
per parameter set, one chain per thread:

  stats_L16.json : L = 16, M = 8, g = 0.1, J = 1, K2 = 1, K4 = 0, T = 0.7,
                   8 chains (seeds 0..7) x 2000 sweeps
  stats_L64.json : L = 64, M = 8, g = 0.1, J = 1, K2 = 1.5, K4 = -0.5,
                   T in {0.5, 0.8}, 8 chains (seeds 1..8) x 10^4 sweeps

Each chain starts from the purpose-0 uniform state of its seed, discards the
first 20 % of sweeps and takes one sample per sweep.  Per chain: batch means
(20 batches) of |M|, M_par, M_z, |M_z|, E/N (L = 16 only) and the wall density; the cone
angle of eq. (17) from per-batch accumulators with a jackknife over batches.

usage: python tests/golden/make_golden_stats.py [L16|L64|all]
"""
import concurrent.futures as cf
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402

NBATCH = 20
SCALARS = ("MABS", "MPAR", "MZ", "MZABS", "E", "WALLDENS")


def chain_stats(L, M, p, nsweeps, energy=True):
    burn = nsweeps // 5
    nsamp = nsweeps - burn
    nsamp -= nsamp % NBATCH
    s0 = oracle.init_spins(L, p["seed"], p["replica_id"])
    op = oracle.params(p["T"], p["J"], p["K2"], p["K4"], p["g"], p["seed"], p["replica_id"])
    t0 = time.time()
    r = oracle.run(L, M, op, s0, 0, burn, nsamp, mode="sequential", with_energy=energy, nbatch=NBATCH)
    out = {"seed": p["seed"], "sweeps": nsweeps, "burn": burn, "samples": nsamp,
           "acceptance": r["accepted"] / float((burn + nsamp) * L * L), "cpu_s": time.time() - t0}
    obs = r["obs"]
    for name in SCALARS:
        x = obs[:, oracle.OBS[name]]
        b = x.reshape(NBATCH, -1).mean(axis=1)
        out[name] = {"mean": float(x.mean()), "se": float(b.std(ddof=1) / math.sqrt(NBATCH))}
    acc = r["eta_acc"]                       # [NBATCH][N] sums of (theta - pi/2)^2
    per = nsamp // NBATCH

    def eta_of(sums, n):
        return float(np.mean(np.sqrt((2 / math.pi) ** 2 * sums / n)))

    full = eta_of(acc.sum(axis=0), nsamp)
    jk = np.array([eta_of(acc.sum(axis=0) - acc[b], nsamp - per) for b in range(NBATCH)])
    se = math.sqrt((NBATCH - 1) / NBATCH * np.sum((jk - jk.mean()) ** 2))
    out["ETA"] = {"mean": full, "se": se}
    return out


def combine(chains):
    """Mean over chains with SE = sqrt(sum se_i^2) / n (independent chains)."""
    res = {}
    for name in SCALARS + ("ETA",):
        m = np.array([c[name]["mean"] for c in chains])
        se = np.array([c[name]["se"] for c in chains])
        res[name] = {"mean": float(m.mean()), "se": float(math.sqrt(np.sum(se ** 2)) / len(m)),
                     "chain_spread_se": float(m.std(ddof=1) / math.sqrt(len(m))) if len(m) > 1 else None}
    return res


def run_set(name, L, M, reps, nsweeps, threads, energy=True):
    with cf.ThreadPoolExecutor(threads) as ex:
        chains = list(ex.map(lambda p: chain_stats(L, M, p, nsweeps, energy), reps))
    return {"name": name, "L": L, "M": M, "params": reps[0] | {"seed": None, "replica_id": 0},
            "chains": chains, "combined": combine(chains)}


def main(which):
    threads = max(1, min(8, os.cpu_count() or 1))
    if which in ("L16", "all"):
        reps = [dict(T=0.7, J=1.0, K2=1.0, K4=0.0, g=0.1, seed=s, replica_id=0) for s in range(8)]
        res = run_set("L16_T0.7", 16, 8, reps, 2000, threads)
        json.dump(res, open(os.path.join(HERE, "stats_L16.json"), "w"), indent=1)
        print("L16 done", res["combined"]["MABS"])
    if which in ("L64", "all"):
        out = {}
        # the energy needs a fresh O(N^2) field per sample: not recorded here
        with cf.ThreadPoolExecutor(2) as ex:
            futs = {}
            for T in (0.5, 0.8):
                reps = [dict(T=T, J=1.0, K2=1.5, K4=-0.5, g=0.1, seed=s, replica_id=0) for s in range(1, 9)]
                futs[T] = ex.submit(run_set, "L64_T%.1f" % T, 64, 8, reps, 10000, max(1, threads // 2), False)
            for T, f in futs.items():
                out["T%.1f" % T] = f.result()
                print("L64 T", T, out["T%.1f" % T]["combined"]["MABS"], flush=True)
        json.dump(out, open(os.path.join(HERE, "stats_L64.json"), "w"), indent=1)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "all")
