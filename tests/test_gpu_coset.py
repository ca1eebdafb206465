"""The paper's l-coset simultaneous update (Sec. 3.1) on the GPU against the
oracle: FP64 trajectories and accept counts (1e-12, equal counts) on both
field paths, the l = L limit against exact sequential Metropolis, counters and
argument checks."""
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


def _params(R, T=0.8, g=0.25):
    return [workloads.replica(T * (1 + 0.15 * r), 1.0, 1.2, -0.4, g, seed=70 + r, replica_id=r) for r in range(R)]


def _op(p):
    return oracle.params(p["T"], p["J"], p["K2"], p["K4"], p["g"], p["seed"], p["replica_id"], p["model"])


@pytest.mark.parametrize("algo", ["fft", "direct"])
@pytest.mark.parametrize("L,l", [(8, 2), (16, 4), (16, 2), (32, 8), (24, 3), (24, 6)])
def test_coset_trajectory_fp64(algo, L, l):
    print("coset %s L=%d l=%d" % (algo, L, l), flush=True)
    R, M, nsw = 2, 2, 2
    reps = _params(R)
    W = oracle.lattice_sum_kernel(L, M)
    s0 = workloads.random_spins(L * L, R, 17)
    starts = [5, 300]
    with ddmc.Plan(L, M, R, prec="f64", algo=algo) as plan:
        dp = ddmc.replica_params_upload(reps)
        s = torch.as_tensor(s0.copy()).cuda()
        ctr = torch.tensor(starts, dtype=torch.int64, device="cuda")
        acc = torch.zeros(R, dtype=torch.int64, device="cuda")
        ddmc.metropolis_sweep_coset(plan, R, dp, s, l, ctr, nsw, acc)
        torch.cuda.synchronize()
        sg = s.cpu().numpy().reshape(R, 3, L * L)
        assert ctr.cpu().numpy().tolist() == [v + nsw for v in starts]
        accg = acc.cpu().numpy()
    for r, p in enumerate(reps):
        ref, nacc = oracle.sweep_coset(L, W, _op(p), s0[r], l, starts[r], nsw)
        assert np.abs(sg[r] - ref).max() <= 1e-12
        assert accg[r] == nacc > 0


@pytest.mark.parametrize("L", [8, 64])
def test_coset_of_single_sites_is_exact_metropolis(L):
    """l = L on the FFT path: every coset is one site, so the GPU sweep is the
    oracle's exact sequential Metropolis (incremental exact field) in index
    order.  At L = 64 in FP64 the kernel W does not fit in LDS next to the
    spins and the one-workgroup coset kernel reads it from global memory."""
    print("single-site cosets L=%d" % L, flush=True)
    M, R = 2, 1
    reps = _params(R, T=0.6, g=0.3)
    W = oracle.lattice_sum_kernel(L, M)
    s0 = workloads.random_spins(L * L, R, 23)
    with ddmc.Plan(L, M, R, prec="f64", algo="fft") as plan:
        dp = ddmc.replica_params_upload(reps)
        s = torch.as_tensor(s0.copy()).cuda()
        ctr = torch.tensor([11], dtype=torch.int64, device="cuda")
        acc = torch.zeros(R, dtype=torch.int64, device="cuda")
        ddmc.metropolis_sweep_coset(plan, R, dp, s, L, ctr, 1, acc)
        torch.cuda.synchronize()
        sg = s.cpu().numpy().reshape(3, L * L)
    ref, _, nacc = oracle.sweep_sequential(L, W, _op(reps[0]), s0[0], oracle.field(L, W, s0[0]), 11, 1)
    assert np.abs(sg - ref).max() <= 1e-12
    assert int(acc[0]) == nacc


def test_coset_fp32_matches_fp64_decisions_mostly():
    """FP32 coset sweeps follow the FP64 ones except where a decision lies in
    the rounding band; over one sweep at L = 32 the states agree to FP32
    precision at all but a handful of sites."""
    L, l, R = 32, 4, 2
    reps = _params(R)
    s0 = workloads.random_spins(L * L, R, 31)
    out = {}
    for prec in ("f64", "f32"):
        with ddmc.Plan(L, 4, R, prec=prec, algo="fft") as plan:
            dp = ddmc.replica_params_upload(reps)
            s = torch.as_tensor(s0.astype(np.float32 if prec == "f32" else np.float64)).cuda()
            ctr = torch.zeros(R, dtype=torch.int64, device="cuda")
            ddmc.metropolis_sweep_coset(plan, R, dp, s, l, ctr, 1)
            torch.cuda.synchronize()
            out[prec] = s.double().cpu().numpy()
    diff = np.abs(out["f64"] - out["f32"]).max(axis=1)   # [R][N]
    assert (diff > 1e-4).sum() <= 4, (diff > 1e-4).sum()


def test_coset_small_cosets_fp32_matches_fp64():
    """L = 64, l = 32 (four sites per coset, the paper's demonstration case):
    the one-workgroup kernel with W in LDS (FP32) against the one that reads W
    from global memory (FP64).  Over two sweeps the states agree to FP32
    precision at all but a handful of sites, and the counters advance."""
    L, l, R, nsw = 64, 32, 2, 2
    reps = _params(R)
    s0 = workloads.random_spins(L * L, R, 37)
    out, accs = {}, {}
    for prec in ("f64", "f32"):
        print("coset L=%d l=%d %s" % (L, l, prec), flush=True)
        with ddmc.Plan(L, 2, R, prec=prec, algo="fft") as plan:
            dp = ddmc.replica_params_upload(reps)
            s = torch.as_tensor(s0.astype(np.float32 if prec == "f32" else np.float64)).cuda()
            ctr = torch.tensor([3, 9], dtype=torch.int64, device="cuda")
            acc = torch.zeros(R, dtype=torch.int64, device="cuda")
            ddmc.metropolis_sweep_coset(plan, R, dp, s, l, ctr, nsw, acc)
            torch.cuda.synchronize()
            assert ctr.cpu().tolist() == [3 + nsw, 9 + nsw]
            out[prec] = s.double().cpu().numpy()
            accs[prec] = acc.cpu().numpy()
    diff = np.abs(out["f64"] - out["f32"]).max(axis=1)
    assert (diff > 1e-4).sum() <= 8, (diff > 1e-4).sum()
    n = np.linalg.norm(out["f32"].reshape(R, 3, L * L), axis=1)
    assert np.abs(n - 1).max() < 1e-5
    assert np.all(np.abs(accs["f64"].astype(np.int64) - accs["f32"].astype(np.int64)) <= 8)
    assert np.all(accs["f64"] > 0)


def _f32_move(L, W, op, p, state, k, sweep):
    """The oracle's FP64 dE and decision for site k of `state` with the exact
    field of that state at k, the draws rounded as the FP32 path rounds them
    (u = (floor(x / 2^9) + 1/2) 2^-23); returns the proposed spin, the
    decision and |u - min(1, exp(-dE/T))|."""
    x = oracle.philox4x32_10([k, sweep, p["replica_id"], 1], [p["seed"] & 0xFFFFFFFF, p["seed"] >> 32])
    u0, u1, u2 = (((v >> 9) + 0.5) * 2.0 ** -23 for v in x[:3])
    S = -state[:, k] if p["model"] == 1 else oracle.direction(u0, u1)   # Ising: the reversal
    h = np.zeros((3, L * L))
    h[:, k] = oracle.field_site(L, W, state, k)
    dE = oracle.delta_e(L, W, op, state, h, k, S)
    with np.errstate(over="ignore"):
        pr = min(1.0, float(np.exp(-dE / p["T"])))
    acc = dE <= 0 or u2 < pr
    return S, bool(acc), abs(u2 - pr)


@pytest.mark.parametrize("model", [0, 1])
@pytest.mark.parametrize("L,l", [(64, 32), (16, 4), (24, 6), (48, 16)])
def test_coset_small_cosets_fp32_decisions(L, l, model):
    """The one-workgroup coset kernel in FP32 (trial spins drawn at the start
    of the sweep, the uniform and the site's own terms of dE folded into an
    acceptance threshold there, field kept in FP64 and brought up to date after
    each coset; power-of-two and other L) against the oracle's decisions,
    coset by coset: one sweep from
    a state the kernel has already evolved; the state before coset k is the
    starting state with the sites of cosets 0 .. k-1 taken from the GPU's
    result (each site is proposed once per sweep).  The oracle's dE uses the
    exact field of that state.  Decisions agree wherever |u - exp(-dE/T)|
    exceeds the FP32 band 1e-4; a moved site holds the FP32 proposal.
    Heisenberg (model 0) and dipolar Ising (model 1: the trial is the
    reversal, so only the self-image term of the site's own terms remains)."""
    print("coset fp32 decisions L=%d l=%d model=%d" % (L, l, model), flush=True)
    R, M = 2, 8
    if model == 0:
        reps = _params(R, T=0.7, g=0.3)
    else:
        reps = [workloads.replica(1.2 * (1 + 0.2 * r), 1.0, 0.0, 0.0, 0.6, seed=90 + r, replica_id=r, model=1)
                for r in range(R)]
    N = L * L
    starts = [5, 77]
    with ddmc.Plan(L, M, R, prec="f32", algo="fft") as plan:
        dp = ddmc.replica_params_upload(reps)
        s = plan.spins(R)
        ddmc.init_spins(plan, R, dp, s)
        ctr = torch.tensor(starts, dtype=torch.int64, device="cuda")
        ddmc.metropolis_sweep_coset(plan, R, dp, s, l, ctr, 2)     # leave the uniform start
        torch.cuda.synchronize()
        s0 = s.double().cpu().numpy().reshape(R, 3, N)
        acc = torch.zeros(R, dtype=torch.int64, device="cuda")
        ddmc.metropolis_sweep_coset(plan, R, dp, s, l, ctr, 1, acc)   # the sweep under test
        torch.cuda.synchronize()
        s1 = s.double().cpu().numpy().reshape(R, 3, N)
        accg = acc.cpu().numpy()
    W = oracle.lattice_sum_kernel(L, M)
    per = L // l
    checked = 0
    for r, p in enumerate(reps):
        op = _op(p)
        sweep = starts[r] + 2
        state = s0[r].copy()
        n_acc = n_band = 0
        for k in range(l * l):
            cy, cx = divmod(k, l)
            sites = [(cy + b * l) * L + cx + a * l for b in range(per) for a in range(per)]
            for i in sites:
                S, acc_i, band = _f32_move(L, W, op, p, state, i, sweep)
                moved = np.abs(s1[r][:, i] - S).max() <= 1e-6
                stayed = np.array_equal(s1[r][:, i], state[:, i])
                assert moved or stayed, (r, k, i)
                if band > 1e-4:
                    assert moved == acc_i, (r, k, i, band)
                else:
                    n_band += 1
                n_acc += int(moved and not stayed)
                checked += 1
            state[:, sites] = s1[r][:, sites]
        assert n_acc > 0
        if n_band == 0:
            assert accg[r] == n_acc
    assert checked == R * N


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_coset_small_cosets_calls_and_batching(prec):
    """One workgroup per replica, whole call in one launch: two calls of one
    sweep equal one call of two (the field is recomputed at each call's
    start, so FP64 agrees to rounding and FP32 to its tolerance), a replica
    run alone equals the same replica in a batch bit for bit, and the accept
    counts add up."""
    L, l, R = 16, 4, 3
    reps = _params(R)
    s0 = workloads.random_spins(L * L, R, 41).astype(np.float64 if prec == "f64" else np.float32)
    tol = 1e-12 if prec == "f64" else 1e-5

    def run(idx, calls):
        with ddmc.Plan(L, 2, len(idx), prec=prec, algo="fft") as plan:
            dp = ddmc.replica_params_upload([reps[i] for i in idx])
            s = torch.as_tensor(s0[idx].copy()).cuda()
            ctr = torch.tensor([4] * len(idx), dtype=torch.int64, device="cuda")
            acc = torch.zeros(len(idx), dtype=torch.int64, device="cuda")
            for n in calls:
                ddmc.metropolis_sweep_coset(plan, len(idx), dp, s, l, ctr, n, acc)
            torch.cuda.synchronize()
            assert ctr.cpu().tolist() == [4 + sum(calls)] * len(idx)
            return s.cpu().numpy(), acc.cpu().numpy()

    one, acc1 = run([0, 1, 2], [2])
    two, acc2 = run([0, 1, 2], [1, 1])
    alone, acc_a = run([1], [2])
    assert np.abs(one - two).max() <= tol
    assert np.array_equal(acc1, acc2)
    assert np.array_equal(alone[0], one[1])
    assert acc_a[0] == acc1[1] > 0


@pytest.mark.parametrize("L,l", [(16, 4), (16, 2)])
def test_coset_graph_replay(L, l):
    """A captured coset call (two sweeps, device counters) replayed three times,
    with eager work and synchronizations between the replays, continues the
    chains exactly as eager calls do: the one-workgroup kernel (16, 4) and
    the field-per-coset path (16, 2)."""
    R = 2
    reps = _params(R)
    s0 = workloads.random_spins(L * L, R, 53).astype(np.float32)
    with ddmc.Plan(L, 2, R, prec="f32", algo="fft") as plan:
        dp = ddmc.replica_params_upload(reps)
        s_ref = torch.as_tensor(s0.copy()).cuda()
        ctr_ref = torch.full((R,), 7, dtype=torch.int64, device="cuda")
        acc_ref = torch.zeros(R, dtype=torch.int64, device="cuda")
        refs = []
        for _ in range(3):
            ddmc.metropolis_sweep_coset(plan, R, dp, s_ref, l, ctr_ref, 2, acc_ref)
            torch.cuda.synchronize()
            refs.append((s_ref.cpu().numpy().copy(), acc_ref.cpu().numpy().copy()))
        s = torch.as_tensor(s0.copy()).cuda()
        ctr = torch.full((R,), 7, dtype=torch.int64, device="cuda")
        acc = torch.zeros(R, dtype=torch.int64, device="cuda")
        s_w, ctr_w, acc_w = s.clone(), ctr.clone(), acc.clone()
        ddmc.metropolis_sweep_coset(plan, R, dp, s_w, l, ctr_w, 2, acc_w)   # warm-up on copies
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            ddmc.metropolis_sweep_coset(plan, R, dp, s, l, ctr, 2, acc, torch.cuda.current_stream())
        torch.cuda.synchronize()
        for rep in range(3):
            g.replay()
            torch.cuda.synchronize()
            _ = (s * 2).sum().item()   # eager work between replays
            assert np.array_equal(s.cpu().numpy(), refs[rep][0]), rep
            assert np.array_equal(acc.cpu().numpy(), refs[rep][1]), rep
            assert ctr.cpu().tolist() == [7 + 2 * (rep + 1)] * R
        del g


def test_coset_arguments():
    with ddmc.Plan(16, 2, 1, prec="f32", algo="fft") as plan:
        dp = ddmc.replica_params_upload(_params(1))
        s = plan.spins(1)
        ctr = torch.zeros(1, dtype=torch.int64, device="cuda")
        for bad in (1, 3, 32, 0):
            with pytest.raises(ddmc.DDMCError):
                ddmc.metropolis_sweep_coset(plan, 1, dp, s, bad, ctr, 1)
        ddmc.metropolis_sweep_coset(plan, 1, dp, s, 2, ctr, 0)    # no sweeps: no-op
        assert int(ctr[0]) == 0
