"""Checkerboard sweeps with a whole replica in one workgroup (plans of
DDMC_FIELD_FFT_LDS): every half-sweep's FFT field and colour update run in
LDS for all sweeps of a call, one launch per call, several lattice sizes per
launch (metropolis_sweep_multi).

Against the oracle: FP64 trajectories and accept counts (1e-12, equal counts)
of Heisenberg and Ising replicas; FP32 decisions of both half-sweeps checked
on the same states and draws outside the FP32 band (|u - exp(-dE/T)| > 1e-4),
with the oracle's exact field.  Against the library's other calls: several
sizes in one launch equal each size alone, bit for bit; captured calls replay
like eager ones; device counters and accept counts advance."""
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


def _params(R, T=0.7, g=0.25, seed0=41, model=0):
    return [workloads.replica(T * (1 + 0.1 * r), 1.0, 1.5, -0.5, g, seed=seed0 + 3 * r, replica_id=r + 1,
                              model=model) for r in range(R)]


def _op(p):
    return oracle.params(p["T"], p["J"], p["K2"], p["K4"], p["g"], p["seed"], p["replica_id"], p.get("model", 0))


def _host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


@pytest.mark.parametrize("L", [8, 16, 24, 32, 48])
@pytest.mark.parametrize("model", [0, 1])
def test_lds_trajectory_fp64(L, model):
    print("lds fp64 trajectory L=%d model=%d" % (L, model), flush=True)
    R, M, nsw = 2, 3, 3
    reps = _params(R, model=model)
    W = oracle.lattice_sum_kernel(L, M)
    if model == 1:
        s0 = np.stack([oracle.init_ising(L, p["seed"], p["replica_id"]) for p in reps])
    else:
        s0 = workloads.random_spins(L * L, R, 70 + L)
    starts = [9, 1234]
    with ddmc.Plan(L, M, R, prec="f64", algo="fft_lds") as plan:
        assert plan.algo == "fft_lds"
        dp = ddmc.replica_params_upload(reps)
        s = torch.as_tensor(s0.copy()).cuda()
        ctr = torch.tensor(starts, dtype=torch.int64, device="cuda")
        acc = torch.zeros(R, dtype=torch.int64, device="cuda")
        ddmc.metropolis_sweep_dev(plan, R, dp, s, ctr, nsw, acc)
        sg = _host(s).reshape(R, 3, L * L)
        assert ctr.cpu().tolist() == [v + nsw for v in starts]
        accg = acc.cpu().numpy()
    for r, p in enumerate(reps):
        ref, nacc = oracle.sweep_checkerboard(L, W, _op(p), s0[r], starts[r], nsw)
        assert np.abs(sg[r] - ref).max() <= 1e-12, r
        assert accg[r] == nacc > 0


def _f32_decision(L, W, op, p, state, k, sweep):
    x = oracle.philox4x32_10([k, sweep, p["replica_id"], 1], [p["seed"] & 0xFFFFFFFF, p["seed"] >> 32])
    u0, u1, u2 = (((v >> 9) + 0.5) * 2.0 ** -23 for v in x[:3])
    S = oracle.direction(u0, u1)
    h = np.zeros((3, L * L))
    h[:, k] = oracle.field_site(L, W, state, k)
    dE = oracle.delta_e(L, W, op, state, h, k, S)
    with np.errstate(over="ignore"):
        pr = min(1.0, float(np.exp(-dE / p["T"])))
    return S, bool(dE <= 0 or u2 < pr), abs(u2 - pr)


@pytest.mark.parametrize("L", [16, 48, 64])
def test_lds_decisions_fp32(L):
    """One FP32 sweep (host sweep index) from a state the path has evolved:
    colour 0 is decided on the starting state, colour 1 on the state after
    colour 0 (its colour-0 sites taken from the GPU's result)."""
    print("lds fp32 decisions L=%d" % L, flush=True)
    R, M = 2, 8
    reps = _params(R, T=0.6, g=0.3)
    N = L * L
    with ddmc.Plan(L, M, R, prec="f32", algo="fft_lds") as plan:
        dp = ddmc.replica_params_upload(reps)
        s = plan.spins(R)
        ddmc.init_spins(plan, R, dp, s)
        ddmc.metropolis_sweep(plan, R, dp, s, 100, 3)
        s0 = _host(s).reshape(R, 3, N)
        acc = torch.zeros(R, dtype=torch.int64, device="cuda")
        ddmc.metropolis_sweep(plan, R, dp, s, 103, 1, acc)
        s1 = _host(s).reshape(R, 3, N)
        accg = acc.cpu().numpy()
    W = oracle.lattice_sum_kernel(L, M)
    color_of = (np.arange(N) % L + np.arange(N) // L) % 2
    for r, p in enumerate(reps):
        op = _op(p)
        state = s0[r].copy()
        n_acc = n_band = 0
        for color in (0, 1):
            sites = np.where(color_of == color)[0]
            for k in sites:
                k = int(k)
                S, acc_k, band = _f32_decision(L, W, op, p, state, k, 103)
                moved = np.abs(s1[r][:, k] - S).max() <= 1e-6
                stayed = np.array_equal(s1[r][:, k], state[:, k])
                assert moved or stayed, (r, k)
                if band > 1e-4:
                    assert moved == acc_k, (r, color, k, band)
                else:
                    n_band += 1
                n_acc += int(moved and not stayed)
            state[:, sites] = s1[r][:, sites]
        assert n_acc > 0
        if n_band == 0:
            assert accg[r] == n_acc


def test_lds_multi_equals_each_size_alone():
    """Three lattice sizes (and an empty group) in one launch give every
    replica exactly the chain its own plan's metropolis_sweep_dev gives it."""
    specs = [(32, 3), (64, 2), (48, 2), (16, 0)]
    groups, alone = [], []
    for i, (L, R) in enumerate(specs):
        Rp = max(R, 1)
        plan = ddmc.Plan(L, 4, Rp, prec="f32", algo="fft_lds")
        reps = _params(Rp, T=0.5 + 0.1 * i, g=0.2, seed0=300 + 10 * i)
        dp = ddmc.replica_params_upload(reps)
        s = plan.spins(Rp)
        ddmc.init_spins(plan, Rp, dp, s)
        ctr = torch.arange(Rp, dtype=torch.int64, device="cuda") * 5 + i
        acc = torch.zeros(Rp, dtype=torch.int64, device="cuda")
        s2, ctr2, acc2 = s.clone(), ctr.clone(), acc.clone()
        groups.append((plan, R, dp, s, ctr, acc))
        alone.append((plan, R, dp, s2, ctr2, acc2))
    ddmc.metropolis_sweep_multi(groups, 4)
    for plan, R, dp, s2, ctr2, acc2 in alone:
        ddmc.metropolis_sweep_dev(plan, R, dp, s2, ctr2, 4, acc2)
    torch.cuda.synchronize()
    for (plan, R, _, s, ctr, acc), (_, _, _, s2, ctr2, acc2) in zip(groups, alone):
        assert torch.equal(s, s2) and torch.equal(ctr, ctr2) and torch.equal(acc, acc2), plan.L
        if R:
            assert acc.min().item() > 0
        plan.close()


def test_lds_graph_replay_and_batch_independence():
    """A captured call replayed three times continues the chains exactly like
    three eager calls, and a replica's chain does not depend on its batch."""
    L, R, G = 64, 4, 5
    reps = _params(R, g=0.2)
    with ddmc.Plan(L, 4, R, prec="f32", algo="fft_lds") as plan:
        dp = ddmc.replica_params_upload(reps)
        s0 = plan.spins(R)
        ddmc.init_spins(plan, R, dp, s0)
        s_ref, c_ref = s0.clone(), torch.zeros(R, dtype=torch.int64, device="cuda")
        refs = []
        for _ in range(3):
            ddmc.metropolis_sweep_dev(plan, R, dp, s_ref, c_ref, G)
            refs.append(_host(s_ref).copy())
        s, c = s0.clone(), torch.zeros(R, dtype=torch.int64, device="cuda")
        sw, cw = s.clone(), c.clone()
        ddmc.metropolis_sweep_dev(plan, R, dp, sw, cw, G)       # warm-up on copies
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            ddmc.metropolis_sweep_dev(plan, R, dp, s, c, G)
        for k in range(3):
            g.replay()
            torch.cuda.synchronize()
            _ = (s * 2).sum().item()
            assert np.array_equal(_host(s), refs[k]), k
        assert c.cpu().tolist() == [3 * G] * R
        # replica 2 alone
        dp1 = ddmc.replica_params_upload([reps[2]])
        s1 = s0[2:3].clone()
        c1 = torch.zeros(1, dtype=torch.int64, device="cuda")
        ddmc.metropolis_sweep_dev(plan, 1, dp1, s1, c1, 3 * G)
        assert np.array_equal(_host(s1)[0], refs[2][2])


def test_lds_argument_checks():
    with pytest.raises(ddmc.DDMCError) as e:
        ddmc.Plan(128, 4, 2, prec="f32", algo="fft_lds")
    assert e.value.status == ddmc.EUNSUPPORTED
    with pytest.raises(ddmc.DDMCError):
        ddmc.Plan(64, 4, 2, prec="f64", algo="fft_lds")
    with pytest.raises(ddmc.DDMCError):
        ddmc.Plan(20, 4, 2, prec="f32", algo="fft_lds")
    with ddmc.Plan(32, 4, 2, prec="f32", algo="fft") as p_fft, \
            ddmc.Plan(32, 4, 2, prec="f32", algo="fft_lds") as p32, \
            ddmc.Plan(16, 4, 2, prec="f64", algo="fft_lds") as p64:
        dp = ddmc.replica_params_upload(_params(2))
        c = torch.zeros(2, dtype=torch.int64, device="cuda")
        with pytest.raises(ddmc.DDMCError):     # not an LDS plan
            ddmc.metropolis_sweep_multi([(p_fft, 2, dp, p_fft.spins(2), c, None)], 1)
        with pytest.raises(ddmc.DDMCError):     # mixed precisions
            ddmc.metropolis_sweep_multi([(p32, 2, dp, p32.spins(2), c, None), (p64, 2, dp, p64.spins(2), c, None)], 1)
        dp3 = ddmc.replica_params_upload(_params(3))
        with pytest.raises(ddmc.DDMCError):     # R above R_max
            ddmc.metropolis_sweep_multi([(p32, 3, dp3, torch.zeros(3 * 3 * 32 * 32, device="cuda"),
                                          torch.zeros(3, dtype=torch.int64, device="cuda"), None)], 1)


def test_tuner_times_sampled_steps():
    """tune.pick(sampled=True) times both forms on sampled steps
    (metropolis_sample) and keeps that record apart from the plain one."""
    from paper_1211_6234_amd import tune
    print("tuner, sampled steps", flush=True)
    form = tune.pick(32, 4, "f32", sweeps=4, reps=1, sampled=True)
    rec = tune.report()[(32, 4, "f32", "sampled")]
    assert form == rec["form"] and set(rec["ms_per_sweep"]) == {"auto", "fft_lds"}
    assert form == min(rec["ms_per_sweep"], key=rec["ms_per_sweep"].get)
    assert all(v > 0 for v in rec["ms_per_sweep"].values())
    assert (32, 4, "f32") not in tune.report() or tune.report()[(32, 4, "f32")] is not rec
