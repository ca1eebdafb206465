"""Failure detection on the device: NaN and infinite spin components written
into a state (the injection is done by the host into the spin array, not by a
kernel) are counted by the observables' health slot on every path that sums
observables, and a Metropolis update never accepts a move whose energy change
is NaN.

Paths: `observables` with and without a field (direct and FFT plans, FP32 and
FP64), and the fused sampling sweep of the FFT path (`metropolis_sample`: the
colour-0 row kernel sums the sample, the final-state sample a separate row
pass).  A NaN spin component spreads into the field of every site through the
convolution, so every energy change of the sweep is NaN: the call must accept
nothing and leave every healthy spin as it was."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1211_6234_amd import ddmc, workloads

pytestmark = pytest.mark.gpu

BAD = [(0, 3, float("nan")), (2, 17, float("inf")), (1, 40, float("-inf")), (0, 55, float("nan")),
       (2, 55, float("inf"))]   # (component, site, value): four sites


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ddmc.lib()
    oracle.build()


def _state(L, R, prec, seed=11):
    s = workloads.random_spins(L * L, R, seed).reshape(R, 3, L * L)
    for c, i, v in BAD:
        s[0, c, i] = v
    dt = torch.float64 if prec == "f64" else torch.float32
    return s, torch.as_tensor(s.reshape(-1)).to(dt).cuda()


def _params(R):
    return [workloads.replica(0.8, 1.0, 1.2, -0.3, 0.2, seed=3 + r, replica_id=r + 1) for r in range(R)]


@pytest.mark.parametrize("algo,prec", [("direct", "f32"), ("direct", "f64"), ("fft", "f32"), ("fft", "f64")])
def test_observables_count_nonfinite_sites(algo, prec):
    print("nonfinite observables %s %s" % (algo, prec), flush=True)
    L, R = 8, 2
    s_host, s = _state(L, R, prec)
    reps = _params(R)
    with ddmc.Plan(L, 2, R, prec=prec, algo=algo) as plan:
        dp = ddmc.replica_params_upload(reps)
        h = plan.spins(R)
        ddmc.local_field(plan, R, s, h)
        for hh in (h, None):
            out = torch.zeros((R, ddmc.NOBS), dtype=torch.float64, device="cuda")
            ddmc.observables(plan, R, dp, s, hh, out, None)
            o = out.cpu().numpy()
            assert o[0, ddmc.OBS["NONFINITE"]] == 4.0 and o[1, ddmc.OBS["NONFINITE"]] == 0.0
            assert math.isnan(o[0, ddmc.OBS["MX"]]) and np.isfinite(o[1, ddmc.OBS["MX"]])
            if hh is not None:
                assert math.isnan(o[0, ddmc.OBS["E"]]) and np.isfinite(o[1, ddmc.OBS["E"]])
    ref = oracle.observables(L, None, oracle.params(**{k: reps[0][k] for k in ("T", "J", "K2", "K4", "g")}),
                             s_host[0])
    assert ref[oracle.OBS["NONFINITE"]] == 4.0


@pytest.mark.parametrize("algo", ["fft", "fft_lds"])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_sample_counts_and_rejects_nan_moves(prec, algo):
    """Two sampled sweeps of the FFT path (four launches per sweep, or one
    workgroup per replica) on a batch whose replica 0 carries the injected
    components: both samples count 4 sites for replica 0 and 0 for replica 1,
    replica 0 accepts no move (every energy change is NaN) and keeps its
    state, replica 1 evolves normally."""
    print("nonfinite sample %s %s" % (prec, algo), flush=True)
    L, R = 16, 2
    s_host, s = _state(L, R, prec, seed=12)
    reps = _params(R)
    with ddmc.Plan(L, 2, R, prec=prec, algo=algo) as plan:
        dp = ddmc.replica_params_upload(reps)
        s0 = s.clone()
        ctr = torch.zeros(R, dtype=torch.int64, device="cuda")
        acc = torch.zeros(R, dtype=torch.int64, device="cuda")
        obs = torch.zeros((2, R, ddmc.NOBS), dtype=torch.float64, device="cuda")
        ddmc.metropolis_sample(plan, R, dp, s, ctr, 2, obs, None, acc)
        torch.cuda.synchronize()
        o = obs.cpu().numpy()
        assert (o[:, 0, ddmc.OBS["NONFINITE"]] == 4.0).all() and (o[:, 1, ddmc.OBS["NONFINITE"]] == 0.0).all()
        a = acc.cpu().numpy()
        assert a[0] == 0 and a[1] > 0
        n = 3 * L * L
        before, after = s0.double().cpu().numpy(), s.double().cpu().numpy()
        assert np.array_equal(np.isnan(after[:n]), np.isnan(before[:n]))
        assert np.array_equal(after[:n][np.isfinite(before[:n])], before[:n][np.isfinite(before[:n])])
        assert not np.array_equal(after[n:], before[n:])
