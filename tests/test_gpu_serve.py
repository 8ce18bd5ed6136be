"""GPU test of the serving loop: Poisson arrivals from 16 client threads
into the background scheduler under a memory budget that binds; every
instance's output must equal, bit for bit, the same instance run alone, and
the admitted footprint must never exceed the budget, nor the device memory
the requests allocate."""
import pytest
import torch

from paper_1303_5164_amd import serve as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def server():
    srv = S.Server(0, base_scale=1 / 64)
    srv.references(reps=2)
    return srv


@pytest.mark.parametrize("policy", ["fifo", "markov"])
def test_serving_outputs_match_solo_and_budget_holds(server, policy):
    n = 240
    rate = 0.9 / (server.mean_service_ms() / 1e3)
    reqs = S.arrivals(5, n, rate, clients=16)
    insts = {}
    for k in server.kinds:
        for c in S.SIZE_LOG2:
            insts[k, c] = server.new_instance(k, c).footprint
    budget = 2 * max(insts.values())
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    recs, summ = server.serve(reqs, policy, budget=budget, verify_every=1)
    # the requests' own allocations stay within the budget (the comparison
    # with the solo output allocates one byte per element of the largest
    # result for a moment)
    slack = max(t.numel() for t in server.ref.values())
    assert torch.cuda.max_memory_allocated() - base <= budget + slack
    assert 0 < summ["allocated_peak_bytes"] <= budget
    print(summ, flush=True)
    assert len(recs) == n and summ["verified"] == n and summ["mismatches"] == 0
    assert 0 < summ["resident_peak_bytes"] <= budget
    assert all(r["done_ns"] >= r["start_ns"] >= r["submit_ns"] for r in recs)
    assert summ["p99_turnaround_ms"] >= summ["p50_turnaround_ms"] > 0
    # instances whose footprints together exceed the budget never ran at once
    ev = sorted([(r["start_ns"], r["footprint"]) for r in recs] +
                [(r["done_ns"], -r["footprint"]) for r in recs])
    live = 0
    for _, f in ev:
        live += f
        assert live <= budget
