"""Dipolar Ising replicas (the appendix on the dipolar Ising model) on the GPU:
initial states, FP64 trajectories on both field paths and both schedules
against the oracle (1e-12, equal accept counts), the stripe order parameters,
Ising and Heisenberg replicas mixed in one launch, and exact Metropolis
(the l = L coset schedule) against the exact 4 x 4 enumeration within 3 sigma."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1211_6234_amd import ddmc, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ddmc.lib()
    oracle.build()


def _ising(R, T=1.2, g=0.6, seed0=40):
    return [workloads.replica(T * (1 + 0.2 * r), 1.0, 0.0, 0.0, g, seed=seed0 + r, replica_id=r, model=1)
            for r in range(R)]


def _op(p):
    return oracle.params(p["T"], p["J"], p["K2"], p["K4"], p["g"], p["seed"], p["replica_id"], p["model"])


def _host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_ising_initial_states(prec):
    L, R = 16, 3
    reps = _ising(R)
    with ddmc.Plan(L, 2, R, prec=prec, algo="fft") as plan:
        dp = ddmc.replica_params_upload(reps)
        s = plan.spins(R)
        ddmc.init_spins(plan, R, dp, s)
        sg = _host(s).reshape(R, 3, L * L)
    for r, p in enumerate(reps):
        assert np.array_equal(sg[r], oracle.init_ising(L, p["seed"], p["replica_id"]))


@pytest.mark.parametrize("algo", ["fft", "direct"])
@pytest.mark.parametrize("schedule", ["checkerboard", "coset"])
def test_ising_trajectory_fp64(algo, schedule):
    L, R, M, nsw = 16, 2, 2, 3
    reps = _ising(R, T=1.0, g=1.5)
    W = oracle.lattice_sum_kernel(L, M)
    with ddmc.Plan(L, M, R, prec="f64", algo=algo) as plan:
        dp = ddmc.replica_params_upload(reps)
        s = plan.spins(R)
        ddmc.init_spins(plan, R, dp, s)
        s0 = _host(s).reshape(R, 3, L * L)
        acc = torch.zeros(R, dtype=torch.int64, device="cuda")
        ctr = torch.tensor([9, 9], dtype=torch.int64, device="cuda")
        if schedule == "checkerboard":
            ddmc.metropolis_sweep_dev(plan, R, dp, s, ctr, nsw, acc)
        else:
            ddmc.metropolis_sweep_coset(plan, R, dp, s, 4, ctr, nsw, acc)
        sg = _host(s).reshape(R, 3, L * L)
        accg = acc.cpu().numpy()
    for r, p in enumerate(reps):
        if schedule == "checkerboard":
            ref, nacc = oracle.sweep_checkerboard(L, W, _op(p), s0[r], 9, nsw)
        else:
            ref, nacc = oracle.sweep_coset(L, W, _op(p), s0[r], 4, 9, nsw)
        assert np.array_equal(sg[r], ref)          # +-1 spins: exact
        assert accg[r] == nacc > 0


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_stripe_observables(prec):
    L, R = 16, 2
    reps = _ising(R)
    N = L * L
    y, x = np.arange(N) // L, np.arange(N) % L
    states = np.zeros((R, 3, N))
    states[0, 2] = np.where(y % 2 == 0, 1.0, -1.0) * np.where(np.arange(N) % 7 == 0, -1.0, 1.0)
    states[1, 2] = np.where(x % 2 == 0, 1.0, -1.0) * np.where(np.arange(N) % 5 == 0, -1.0, 1.0)
    with ddmc.Plan(L, 2, R, prec=prec, algo="fft") as plan:
        dp = ddmc.replica_params_upload(reps)
        s = torch.as_tensor(states.astype(np.float64 if prec == "f64" else np.float32)).cuda()
        out = torch.zeros((R, ddmc.NOBS), dtype=torch.float64, device="cuda")
        ddmc.observables(plan, R, dp, s, None, out)
        og = _host(out)
    for r, p in enumerate(reps):
        ref = oracle.observables(L, None, _op(p), states[r])
        for k in ("MSTH", "MSTV", "MZ", "NH", "NV"):
            assert og[r, ddmc.OBS[k]] == ref[oracle.OBS[k]], k


def test_mixed_models_in_one_launch():
    """A batch of Heisenberg and Ising replicas: each follows the trajectory it
    has alone."""
    L, M = 32, 4
    reps = [workloads.replica(0.9, 1.0, 1.0, 0.0, 0.2, seed=1, replica_id=0),
            workloads.replica(1.1, 1.0, 0.0, 0.0, 0.8, seed=2, replica_id=1, model=1),
            workloads.replica(0.6, 1.0, 1.5, -0.5, 0.1, seed=3, replica_id=2)]
    with ddmc.Plan(L, M, 3, prec="f32", algo="fft") as plan:
        dp = ddmc.replica_params_upload(reps)
        s = plan.spins(3)
        ddmc.init_spins(plan, 3, dp, s)
        s_alone = s.clone()
        ddmc.metropolis_sweep(plan, 3, dp, s, 0, 4)
        batch = _host(s)
        for r in range(3):
            d1 = ddmc.replica_params_upload([reps[r]])
            s1 = s_alone[r:r + 1].clone()
            ddmc.metropolis_sweep(plan, 1, d1, s1, 0, 4)
            assert np.array_equal(_host(s1)[0], batch[r]), r
    assert set(np.unique(batch[1, 2])) <= {-1.0, 1.0} and np.abs(batch[1, :2]).max() == 0.0


def test_exact_metropolis_against_enumeration():
    """The l = L coset schedule is exact sequential Metropolis: on the GPU its
    averages of E, |m| and m_st at L = 4 (16 replicas, direct FP64 field) match
    the exact enumeration of all 65536 states within 3 sigma, and so does the
    staggered susceptibility of its samples (the oracle's estimator)."""
    L, M, R, nsw, burn = 4, 2, 16, 6000, 200
    g, T = 2.5, 1.0
    W = oracle.lattice_sum_kernel(L, M)
    N = L * L
    idx = np.arange(N)
    xs, ys = idx % L, idx // L
    ix, iy = ys * L + (xs + 1) % L, ((ys + 1) % L) * L + xs
    D = W[3][(ys[:, None] - ys[None, :]) % L, (xs[:, None] - xs[None, :]) % L]
    st = ((np.arange(2 ** N)[:, None] >> idx[None, :]) & 1) * 2.0 - 1.0
    E = -(st * (st[:, ix] + st[:, iy])).sum(1) + 0.5 * g * np.einsum("si,ij,sj->s", st, D, st)
    mst = np.hypot((st * np.where(ys % 2 == 0, 1.0, -1.0)).mean(1), (st * np.where(xs % 2 == 0, 1.0, -1.0)).mean(1))
    w = np.exp(-(E - E.min()) / T)
    w /= w.sum()
    exact = {"e": (w * E).sum() / N, "mabs": (w * np.abs(st.mean(1))).sum(), "mst": (w * mst).sum()}
    chi_exact = N / T * ((w * mst * mst).sum() - exact["mst"] ** 2)
    reps = [workloads.replica(T, 1.0, 0.0, 0.0, g, seed=500 + r, replica_id=r, model=1) for r in range(R)]
    with ddmc.Plan(L, M, R, prec="f64", algo="direct") as plan:
        dp = ddmc.replica_params_upload(reps)
        s = plan.spins(R)
        h = plan.spins(R)
        ddmc.init_spins(plan, R, dp, s)
        ctr = torch.zeros(R, dtype=torch.int64, device="cuda")
        ddmc.metropolis_sweep_coset(plan, R, dp, s, L, ctr, burn)
        out = torch.zeros((nsw, R, ddmc.NOBS), dtype=torch.float64, device="cuda")
        for k in range(nsw):
            ddmc.metropolis_sweep_coset(plan, R, dp, s, L, ctr, 1)
            ddmc.local_field(plan, R, s, h, -1)
            ddmc.observables(plan, R, dp, s, h, out[k])
        og = _host(out)
    O = ddmc.OBS
    series = {"e": og[:, :, O["E"]], "mabs": np.abs(og[:, :, O["MZ"]]),
              "mst": np.hypot(og[:, :, O["MSTH"]], og[:, :, O["MSTV"]])}
    for key, v in series.items():
        chain_means = v.reshape(20, nsw // 20, R).mean(axis=1).reshape(-1)    # batch means of every chain
        se = chain_means.std(ddof=1) / math.sqrt(len(chain_means))
        assert abs(v.mean() - exact[key]) <= 3 * se, (key, v.mean(), exact[key], se)
    # the staggered susceptibility of the appendix, one value per chain and batch
    chis = np.array([oracle.staggered_susceptibility(L, T, b[:, r]) for b in og.reshape(20, nsw // 20, R, -1)
                     for r in range(R)])
    chi = np.mean([oracle.staggered_susceptibility(L, T, og[:, r]) for r in range(R)])
    assert abs(chi - chi_exact) <= 3 * chis.std(ddof=1) / math.sqrt(len(chis)), (chi, chi_exact)
