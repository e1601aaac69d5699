"""Scheduling logic of the continuous-batching loop, on the host (FakeEngine)."""
import pytest

from paper_2512_23116_amd import serving
from paper_2512_23116_amd.serving import FakeEngine, Request, serve


def _req(rid, N, arrival, steps=128):
    return Request(rid=rid, N=N, C=0.1, tau0=0.51, force_seed=rid, init_seed=rid,
                   arrival=arrival, steps=steps)


def test_all_requests_complete_and_latencies_are_ordered():
    reqs = [_req(i, 16 + 8 * (i % 3), 0.0005 * i, steps=100 + 7 * i) for i in range(20)]
    eng = FakeEngine(rate=5e9, steps_per_graph=16)
    res = serve(reqs, eng, max_slots=4, hbm_budget=1e12)
    assert res["failed"] == 0 and res["n"] == 20
    for r in reqs:
        assert r.done_steps == r.steps
        assert r.arrival <= r.admit <= r.complete
    assert res["p50_s"] <= res["p99_s"]
    # never more than max_slots lattices in one call, never more steps than a graph
    for call in eng.calls:
        assert len(call) <= 4
        assert all(0 < s <= 16 for _, s in call)
    # every request got exactly its steps
    got = {}
    for call in eng.calls:
        for rid, s in call:
            got[rid] = got.get(rid, 0) + s
    assert got == {r.rid: r.steps for r in reqs}


def test_late_arrivals_join_running_batches():
    reqs = [_req(0, 32, 0.0, steps=640), _req(1, 32, 0.002, steps=64)]
    eng = FakeEngine(rate=2e9, steps_per_graph=64)
    serve(reqs, eng, max_slots=4, hbm_budget=1e12)
    mixed = [c for c in eng.calls if len(c) == 2]
    assert mixed, "the second request never shared a call with the first"
    assert reqs[1].complete < reqs[0].complete


def test_hbm_budget_forces_queueing():
    reqs = [_req(i, 32, 0.0, steps=64) for i in range(4)]
    one = reqs[0].state_bytes
    eng = FakeEngine(rate=1e10, steps_per_graph=64)
    res = serve(reqs, eng, max_slots=16, hbm_budget=2 * one)
    assert max(len(c) for c in eng.calls) == 2
    assert all(r.done_steps == 64 for r in reqs)
    # half the requests waited for memory: the latency splits into queueing + service
    assert res["wait_p50_s"] >= 0 and res["wait_p99_s"] > 0
    assert res["service_p99_s"] > 0
    for r in reqs:
        assert abs((r.admit - r.arrival) + (r.complete - r.admit) - r.latency) < 1e-12


def test_oversized_and_failing_requests_fail_alone():
    reqs = [_req(0, 32, 0.0), _req(1, 200, 0.0), _req(2, 16, 0.0), _req(3, 16, 0.0)]
    eng = FakeEngine(rate=1e10, steps_per_graph=32, fail_rids={2})
    res = serve(reqs, eng, max_slots=4, hbm_budget=reqs[0].state_bytes * 2)
    assert reqs[1].error and reqs[2].error
    assert reqs[0].error is None and reqs[3].error is None
    assert reqs[0].done_steps == reqs[0].steps and reqs[3].done_steps == reqs[3].steps
    assert res["failed"] == 2


def test_request_stream_is_seeded():
    a = serving.make_requests(64, seed=5, rate=2.0)
    b = serving.make_requests(64, seed=5, rate=2.0)
    assert [(r.N, r.C, r.tau0, r.arrival) for r in a] == [(r.N, r.C, r.tau0, r.arrival) for r in b]
    assert {r.N for r in a} <= {32, 48, 64, 96, 128}
    assert all(0.08 <= r.C <= 0.18 and 0.505 <= r.tau0 <= 0.55 for r in a)
    arr = [r.arrival for r in a]
    assert arr == sorted(arr) and arr[-1] == pytest.approx(32.0, rel=0.5)


def test_cache_groups_pack_states_first_fit_decreasing():
    from paper_2512_23116_amd.serving import Request, cache_groups
    mb = 1 << 20
    reqs = [Request(rid=i, N=n, C=0.1, tau0=0.51, force_seed=i, init_seed=i, arrival=0.0)
            for i, n in enumerate([32, 128, 96, 64, 128, 48, 96])]
    steps = [64, 64, 8, 64, 64, 64, 64]
    groups = cache_groups(reqs, steps, 192 * mb)
    # every pair appears once, with its steps
    flat = sorted((r.rid, s) for g in groups for r, s in g)
    assert flat == sorted((r.rid, s) for r, s in zip(reqs, steps))
    for g in groups:
        assert sum(r.state_bytes for r, _ in g) <= 192 * mb
    # largest first: 128^3 (152 MiB) + 64^3 + 48^3 + 32^3, then the other 128^3,
    # then the two 96^3
    assert [[r.N for r, _ in g] for g in groups] == [[128, 64, 48, 32], [128], [96, 96]]
    # no limit: one group in the given order; a state above the limit stands alone
    assert cache_groups(reqs, steps, None) == [list(zip(reqs, steps))]
    assert [len(g) for g in cache_groups(reqs[1:2], steps[1:2], 64 * mb)] == [1]
    assert cache_groups([], [], 192 * mb) == []
