"""Serving: requests of mixed lattice sizes admitted as they arrive, batched
per size with per-request sweep counters; each request's result must be the
same, bit for bit, alone and in the mix (the kernels treat replicas
independently and the sweep index of every move comes from the request's
own counter)."""
import numpy as np
import pytest
import torch

from paper_1211_6234_amd import ddmc, serve, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ddmc.lib()


def _mix():
    specs = [(16, 30), (32, 45), (24, 25), (16, 60), (32, 20), (24, 40), (16, 35)]
    reqs = []
    for i, (L, sweeps) in enumerate(specs):
        p = workloads.replica(0.4 + 0.1 * i, 1.0, 1.0 + 0.2 * i, 0.3 - 0.1 * i, 0.05 + 0.02 * i, seed=100 + i)
        reqs.append(serve.Request(i, L, p, sweeps, arrival=0.0))
    return reqs


def _serve(reqs, chunk):
    srv = serve.Server(hbm_budget_bytes=1 << 30, M=4, prec="f32", slots_per_size=8, chunk_sweeps=chunk,
                       keep_state=True)
    done = srv.run(reqs, realtime=False)
    srv.close()
    return {r.rid: r for r in done}


def test_alone_equals_mixed():
    mixed = _serve(_mix(), chunk=7)
    assert sorted(mixed) == list(range(7))
    for r in _mix():
        alone = _serve([r], chunk=13)[r.rid]
        m = mixed[r.rid]
        assert np.array_equal(alone.state, m.state), r.rid
        assert np.array_equal(alone.result, m.result, equal_nan=True), r.rid
        assert alone.accepted == m.accepted, r.rid
        assert m.done_sweeps == r.sweeps


def test_admission_respects_budget():
    """Room for one L = 32 request: admissions are serialized; a request that
    can never fit is rejected instead of blocking the queue."""
    reqs = [serve.Request(i, 32, workloads.replica(0.7, seed=i), 15 + 5 * i) for i in range(4)]
    reqs.append(serve.Request(9, 64, workloads.replica(0.7, seed=9), 10))
    srv = serve.Server(hbm_budget_bytes=serve.slot_bytes(32) + 10, M=4, slots_per_size=8, chunk_sweeps=10)
    done = srv.run(reqs, realtime=False)
    srv.close()
    by = {r.rid: r for r in done}
    assert by[9].result is None
    served = [by[i] for i in range(4)]
    assert all(r.result is not None and r.done_sweeps == r.sweeps for r in served)
    spans = sorted((r.t_admit, r.t_done) for r in served)
    for (a0, d0), (a1, d1) in zip(spans, spans[1:]):
        assert a1 >= d0 - 1e-9
