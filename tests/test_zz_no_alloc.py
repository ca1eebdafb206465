"""observables_noalloc (the entry point for callers that cannot allocate)
against observables of a plan: the same outputs and cone-angle accumulators
bit for bit, on two calls in a row through the C ABI, the second with fewer
replicas on a smaller lattice, in both precisions; sizes beyond the static
scratch are rejected."""
import numpy as np
import pytest
import torch

from paper_1211_6234_amd import ddmc, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ddmc.lib()


def _case(L, R, prec, seed):
    reps = [workloads.replica(0.5 + 0.1 * r, 1.0, 1.5, -0.5, 0.2, seed=seed + r, replica_id=r) for r in range(R)]
    with ddmc.Plan(L, 4, R, prec=prec, algo="auto") as plan:
        dp = ddmc.replica_params_upload(reps)
        s = plan.spins(R)
        ddmc.init_spins(plan, R, dp, s)
        ddmc.metropolis_sweep(plan, R, dp, s, 3, 2)
        h = plan.spins(R)
        ddmc.local_field(plan, R, s, h, -1)
        eta0 = torch.rand((R, L * L), dtype=torch.float64, device="cuda")
        ref_out = torch.full((R, ddmc.NOBS), float("nan"), dtype=torch.float64, device="cuda")
        ref_eta = eta0.clone()
        ddmc.observables(plan, R, dp, s, h, ref_out, ref_eta)
        out = torch.full((R, ddmc.NOBS), float("nan"), dtype=torch.float64, device="cuda")
        eta = eta0.clone()
        ddmc.observables_noalloc(L, R, dp, s, h, out, eta)
        out_noh = torch.full((R, ddmc.NOBS), float("nan"), dtype=torch.float64, device="cuda")
        ddmc.observables_noalloc(L, R, dp, s, None, out_noh, None)
        ref_noh = torch.full((R, ddmc.NOBS), float("nan"), dtype=torch.float64, device="cuda")
        ddmc.observables(plan, R, dp, s, None, ref_noh, None)
        torch.cuda.synchronize()
        assert torch.equal(out.isnan(), ref_out.isnan())
        assert np.array_equal(out.cpu().numpy(), ref_out.cpu().numpy(), equal_nan=True)
        assert torch.equal(eta, ref_eta)
        assert np.array_equal(out_noh.cpu().numpy(), ref_noh.cpu().numpy(), equal_nan=True)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_noalloc_equals_observables_two_calls(prec):
    print("observables_noalloc %s" % prec, flush=True)
    _case(64, 24, prec, 11)       # first call
    _case(20, 3, prec, 40)        # second call: fewer replicas, smaller lattice


def test_noalloc_rejects_sizes_beyond_its_scratch():
    L, R = 8, ddmc.NOALLOC_R_MAX + 1
    s = torch.zeros((R, 3, L, L), dtype=torch.float32, device="cuda")
    out = torch.zeros((R, ddmc.NOBS), dtype=torch.float64, device="cuda")
    dp = torch.zeros(R * ddmc.PARAMS_BYTES, dtype=torch.uint8, device="cuda")
    with pytest.raises(ddmc.DDMCError) as e:
        ddmc.observables_noalloc(L, R, dp, s, None, out)
    assert e.value.status == ddmc.EINVAL
    with pytest.raises(ddmc.DDMCError):
        ddmc.observables_noalloc(0, 1, dp, s, None, out)
