"""Replica exchange on the GPU (parallel_tempering_swap): decisions and
exchanged states against the oracle's exchange step on the same states,
graph replays, and exact per-temperature averages of a small Ising ladder
(exact Metropolis sweeps + exchanges) against enumeration within 3 sigma."""
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


def _op(p):
    return oracle.params(p["T"], p["J"], p["K2"], p["K4"], p["g"], p["seed"], p["replica_id"], p["model"])


def _host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


@pytest.mark.parametrize("parity", [0, 1])
def test_exchange_matches_oracle(parity):
    L, M, R = 16, 2, 7
    reps = [workloads.replica(0.4 + 0.05 * r, 1.0, 1.0, 0.0, 0.2, seed=200 + r, replica_id=r) for r in range(R)]
    W = oracle.lattice_sum_kernel(L, M)
    s0 = workloads.random_spins(L * L, R, 8)
    # give neighbouring states close energies so that both outcomes occur
    for r in range(1, R, 2):
        s0[r] = s0[r - 1][:, np.random.default_rng(r).permutation(L * L)]
    rounds = np.arange(R) * 13 + 5
    with ddmc.Plan(L, M, R, prec="f64", algo="fft") as plan:
        dp = ddmc.replica_params_upload(reps)
        s = torch.as_tensor(s0.copy()).cuda()
        h = plan.spins(R)
        ddmc.local_field(plan, R, s, h, -1)
        obs = torch.zeros((R, ddmc.NOBS), dtype=torch.float64, device="cuda")
        ddmc.observables(plan, R, dp, s, h, obs)
        ctr = torch.as_tensor(rounds.astype(np.int64)).cuda()
        sw = torch.zeros(R, dtype=torch.int64, device="cuda")
        ddmc.parallel_tempering_swap(plan, R, dp, s, obs, ctr, parity, sw)
        sg, swg = _host(s).reshape(R, 3, L * L), sw.cpu().numpy()
    E = np.array([oracle.energy(L, W, _op(p), s0[r])["total"] for r, p in enumerate(reps)])
    ref = s0.copy()
    swr = np.zeros(R, dtype=np.uint64)
    oracle.pt_swap(L, [_op(p) for p in reps], ref, E, rounds, parity, swr)
    # decisions whose uniform lies within 1e-9 of the threshold may differ by rounding
    for r in range(parity, R - 1, 2):
        d = (1 / reps[r]["T"] - 1 / reps[r + 1]["T"]) * (E[r] - E[r + 1])
        u = oracle.draw(reps[r]["seed"], reps[r]["replica_id"], int(rounds[r]), r, 2)[0]
        if d < 0 and abs(u - math.exp(d)) < 1e-9:
            continue
        assert swg[r] == swr[r], r
        assert np.array_equal(sg[r], ref[r]) and np.array_equal(sg[r + 1], ref[r + 1]), r
    assert swr.sum() > 0


def test_exchange_graph_replay():
    """sample + exchange (both parities) captured once and replayed equals the
    same eager calls; counters advance, so the draws differ between rounds."""
    L, R = 32, 6
    reps = [workloads.replica(0.5 + 0.1 * r, 1.0, 1.5, 0.0, 0.15, seed=300 + r, replica_id=r) for r in range(R)]
    with ddmc.Plan(L, 4, R, prec="f32", algo="fft") as plan:
        dp = ddmc.replica_params_upload(reps)
        s0 = plan.spins(R)
        ddmc.init_spins(plan, R, dp, s0)

        def rounds(s, ctr, obs, sw, st=None):
            for parity in (0, 1):
                ddmc.metropolis_sample(plan, R, dp, s, ctr, 2, obs, stream=st)
                ddmc.parallel_tempering_swap(plan, R, dp, s, obs[1], ctr, parity, sw, stream=st)

        s_ref, c_ref = s0.clone(), torch.zeros(R, dtype=torch.int64, device="cuda")
        o_ref, w_ref = torch.zeros((2, R, ddmc.NOBS), dtype=torch.float64, device="cuda"), \
            torch.zeros(R, dtype=torch.int64, device="cuda")
        snaps = []
        for _ in range(3):
            rounds(s_ref, c_ref, o_ref, w_ref)
            snaps.append(_host(s_ref).copy())
        s, c = s0.clone(), torch.zeros(R, dtype=torch.int64, device="cuda")
        o, w = torch.zeros((2, R, ddmc.NOBS), dtype=torch.float64, device="cuda"), \
            torch.zeros(R, dtype=torch.int64, device="cuda")
        rounds(s.clone(), c.clone(), o.clone(), w.clone())       # warm-up on copies
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            rounds(s, c, o, w, torch.cuda.current_stream())
        torch.cuda.synchronize()
        for k in range(3):
            g.replay()
            torch.cuda.synchronize()
            _ = (s * 2).sum().item()
            assert np.array_equal(_host(s), snaps[k]), k
        assert np.array_equal(w.cpu().numpy(), w_ref.cpu().numpy())
        assert c.cpu().numpy().tolist() == [12] * R


def test_tempering_keeps_each_temperature_exact():
    """3-temperature Ising ladder at L = 4 (direct FP64 field): exact
    Metropolis sweeps (coset l = L) and an exchange attempt per round; each
    slot's <E> and <m_st> equal the exact enumeration at its temperature
    within 3 sigma, and exchanges happen."""
    L, M, g = 4, 2, 2.0
    Ts = [0.8, 1.4, 2.5]
    R = len(Ts)
    W = oracle.lattice_sum_kernel(L, M)
    N = L * L
    idx = np.arange(N)
    xs, ys = idx % L, idx // L
    ix, iy = ys * L + (xs + 1) % L, ((ys + 1) % L) * L + xs
    D = W[3][(ys[:, None] - ys[None, :]) % L, (xs[:, None] - xs[None, :]) % L]
    st = ((np.arange(2 ** N)[:, None] >> idx[None, :]) & 1) * 2.0 - 1.0
    En = -(st * (st[:, ix] + st[:, iy])).sum(1) + 0.5 * g * np.einsum("si,ij,sj->s", st, D, st)
    mst = np.hypot((st * np.where(ys % 2 == 0, 1.0, -1.0)).mean(1), (st * np.where(xs % 2 == 0, 1.0, -1.0)).mean(1))
    exact = []
    for T in Ts:
        w = np.exp(-(En - En.min()) / T)
        w /= w.sum()
        exact.append(((w * En).sum() / N, (w * mst).sum()))
    reps = [workloads.replica(T, 1.0, 0.0, 0.0, g, seed=700 + r, replica_id=r, model=1) for r, T in enumerate(Ts)]
    nround, burn = 8000, 200
    with ddmc.Plan(L, M, R, prec="f64", algo="direct") as plan:
        dp = ddmc.replica_params_upload(reps)
        s = plan.spins(R)
        h = plan.spins(R)
        ddmc.init_spins(plan, R, dp, s)
        ctr = torch.zeros(R, dtype=torch.int64, device="cuda")
        sw = torch.zeros(R, dtype=torch.int64, device="cuda")
        out = torch.zeros((nround, R, ddmc.NOBS), dtype=torch.float64, device="cuda")
        for k in range(nround):
            ddmc.metropolis_sweep_coset(plan, R, dp, s, L, ctr, 1)
            ddmc.local_field(plan, R, s, h, -1)
            ddmc.observables(plan, R, dp, s, h, out[k])
            ddmc.parallel_tempering_swap(plan, R, dp, s, out[k], ctr, k % 2, sw)
        og = _host(out)[burn:]
        swg = sw.cpu().numpy()
    assert swg[0] > 100 and swg[1] > 100
    O = ddmc.OBS
    for r in range(R):
        for key, v in (("e", og[:, r, O["E"]]), ("mst", np.hypot(og[:, r, O["MSTH"]], og[:, r, O["MSTV"]]))):
            n = len(v) // 20 * 20
            b = v[:n].reshape(20, -1).mean(1)
            se = b.std(ddof=1) / math.sqrt(20)
            want = exact[r][0] if key == "e" else exact[r][1]
            assert abs(v.mean() - want) <= 3 * se, (r, key, v.mean(), want, se)


def test_exchanging_ladder_accepts_swaps():
    """The benchmark's exchanging ladder (L = 32, 32 replicas over T in
    [0.6, 1.2]): after 400 sweeps from the uniform start, 50 further rounds of
    10 sampled sweeps and one exchange attempt per pair accept at least one
    swap on every pair and not every attempt overall (an exchange leg that
    moves states, unlike the L = 128 ladder where dBeta dE is far above 1)."""
    w = workloads.ladder_l32_pt(32)
    R, L = len(w["replicas"]), w["L"]
    with ddmc.Plan(L, w["M"], R, prec="f32", algo="fft") as plan:
        dp = ddmc.replica_params_upload(w["replicas"])
        s = plan.spins(R)
        ddmc.init_spins(plan, R, dp, s)
        ctr = torch.zeros(R, dtype=torch.int64, device="cuda")
        obs = torch.zeros((10, R, ddmc.NOBS), dtype=torch.float64, device="cuda")
        sw = torch.zeros(R, dtype=torch.int64, device="cuda")
        for rnd in range(70):
            if rnd == 20:
                sw.zero_()
            ddmc.metropolis_sample(plan, R, dp, s, ctr, 10, obs, None, None)
            ddmc.parallel_tempering_swap(plan, R, dp, s, obs[9], ctr, rnd % 2, sw)
        acc = sw.cpu().numpy()[:R - 1]
    assert (acc >= 1).all(), acc
    assert acc.sum() < 25 * (R - 1), acc
