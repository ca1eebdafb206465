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


def _serve(reqs, chunk, slots=8):
    srv = serve.Server(hbm_budget_bytes=1 << 30, M=4, prec="f32", slots_per_size=slots, chunk_sweeps=chunk,
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


def test_admission_mid_run_equals_alone():
    """Two slots per size for seven requests: later requests are admitted into
    a pool as earlier ones retire, while the other resident request of that
    size is part-way through its sweeps (chunks of 7 sweeps); every result is
    still bit-identical to the request served alone."""
    mixed = _serve(_mix(), chunk=7, slots=2)
    assert sorted(mixed) == list(range(7))
    by_L = {}
    for r in _mix():
        by_L.setdefault(r.L, []).append(r.rid)
    # some request was admitted while another of its size had started and not finished
    overlap = any(mixed[a].t_admit < mixed[b].t_admit < mixed[a].t_done
                  for ids in by_L.values() for a in ids for b in ids if a != b)
    assert overlap
    for r in _mix():
        alone = _serve([r], chunk=13)[r.rid]
        m = mixed[r.rid]
        assert np.array_equal(alone.state, m.state), r.rid
        assert np.array_equal(alone.result, m.result, equal_nan=True), r.rid
        assert alone.accepted == m.accepted, r.rid


def test_admission_does_not_wait_for_a_running_chunk():
    """Admitting into a pool whose chunk is still running only enqueues work
    on the pool's stream: the call returns while the chunk is in flight, and
    the running request's result is unchanged."""
    L = 128
    p0 = workloads.replica(0.6, 1.0, 1.5, 0.0, 0.1, seed=7)
    p1 = workloads.replica(0.9, 1.0, 1.0, 0.2, 0.1, seed=8)
    srv = serve.Server(hbm_budget_bytes=1 << 30, M=4, slots_per_size=4, chunk_sweeps=1500, keep_state=True)
    g = srv._pool_for(L)
    r0 = serve.Request(0, L, p0, 1500)
    g.admit(r0)
    g._graph(1, 1500)                       # capture before timing
    g.run_chunk(1500)
    r1 = serve.Request(1, L, p1, 10)
    g.admit(r1)
    assert not g.done_ev.query(), "the admission waited for the chunk"
    torch.cuda.synchronize()
    state0 = g.s[0].cpu().numpy().copy()
    srv.close()
    alone = _serve([serve.Request(0, L, p0, 1500)], chunk=1500)[0]
    assert np.array_equal(alone.state, state0)


def test_budget_bounds_device_memory():
    """The budget decides the pools' real allocations: with room for three
    L = 32 slots the pool gets three slots, at most three requests are
    resident at once, and the bytes the server holds (torch's tensors of the
    pools and the library's plans, sampled when pools are created) stay
    within the budget."""
    budget = serve.group_bytes(32, 3) + 4096
    assert serve.group_bytes(32, 4) > budget
    reqs = [serve.Request(i, 32, workloads.replica(0.5 + 0.05 * i, seed=i), 12 + 3 * i) for i in range(7)]
    srv = serve.Server(hbm_budget_bytes=budget, M=4, slots_per_size=8, chunk_sweeps=5)
    done = srv.run(reqs, realtime=False)
    assert srv.groups[32].cap == 3
    assert srv.peak_in_use <= budget
    assert 0 < srv.peak_measured <= budget
    srv.close()
    assert all(r.result is not None and r.done_sweeps == r.sweeps for r in done)
    events = sorted([(r.t_admit, 1) for r in done] + [(r.t_done, -1) for r in done])
    live = peak = 0
    for _, d in events:
        live += d
        peak = max(peak, live)
    assert peak <= 3


def test_admission_respects_budget():
    """Room for one L = 32 slot: admissions are serialized; a request that
    can never fit is rejected instead of blocking the queue."""
    reqs = [serve.Request(i, 32, workloads.replica(0.7, seed=i), 15 + 5 * i) for i in range(4)]
    reqs.append(serve.Request(9, 64, workloads.replica(0.7, seed=9), 10))
    srv = serve.Server(hbm_budget_bytes=serve.group_bytes(32, 1) + 10, M=4, slots_per_size=8, chunk_sweeps=10)
    done = srv.run(reqs, realtime=False)
    srv.close()
    by = {r.rid: r for r in done}
    assert by[9].result is None
    served = [by[i] for i in range(4)]
    assert all(r.result is not None and r.done_sweeps == r.sweeps for r in served)
    spans = sorted((r.t_admit, r.t_done) for r in served)
    for (a0, d0), (a1, d1) in zip(spans, spans[1:]):
        assert a1 >= d0 - 1e-9


def test_autotuned_forms_serve_the_same_chains():
    """With the sweep form of each size chosen by measurement, FP64 requests
    follow the same chains as with the fixed forms (both forms are exact to
    rounding in FP64): final states equal to 1e-12."""
    from paper_1211_6234_amd import tune
    specs = [(16, 30), (32, 25), (64, 20)]
    reqs = lambda: [serve.Request(i, L, workloads.replica(0.6 + 0.1 * i, 1.0, 1.2, 0.1, 0.15, seed=200 + i), n)
                    for i, (L, n) in enumerate(specs)]
    out = {}
    for auto in (False, True):
        srv = serve.Server(hbm_budget_bytes=1 << 30, M=4, prec="f64", slots_per_size=4, chunk_sweeps=10,
                           keep_state=True, autotune=auto)
        out[auto] = {r.rid: r for r in srv.run(reqs(), realtime=False)}
        forms = dict(srv.forms)
        srv.close()
    assert set(forms) == {16, 32, 64} and all(f in ("fft_lds", "auto") for f in forms.values())
    assert len(tune.report()) >= 2
    for rid in out[False]:
        assert np.abs(out[False][rid].state - out[True][rid].state).max() <= 1e-12, rid
