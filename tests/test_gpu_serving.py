"""The continuous-batching server: requests arriving while others run are
admitted as memory frees up, every request completes, and each result is
the same (bit for bit) as the request run alone."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage", ["f32", "bf16dev"])
def test_server_results_equal_alone_runs(storage):
    from paper_2102_02655_amd import lbprint as LB
    from paper_2102_02655_amd import serving as S

    reqs = S.make_requests(count=8, seed=11, rate=200.0, lmin=20, lmax=40, steps=30, storage=storage)
    budget = sum(LB.footprint(r.cfg) for r in reqs[:3])  # at most ~3 resident at once
    stats = S.Server(budget, chunk=8, keep_fields=True, lanes=2).run(reqs)
    assert sorted(r.id for r in stats.results) == list(range(8))
    assert stats.peak_bytes <= budget
    by_id = {r.id: r for r in stats.results}
    for req in reqs:
        sim = LB.Sim(req.cfg, req.ry, req.rb)
        sim.step(req.steps)
        ry, rb, u, cons = sim.moments(dtype=np.float64)
        got = by_id[req.id]
        assert np.array_equal(got.fields[0], ry) and np.array_equal(got.fields[1], rb)
        assert np.array_equal(got.fields[2], u)
        assert np.array_equal(got.mass, cons["mass"])
        sim.close()
    s = stats.summary()
    assert s["requests"] == 8 and s["latency_p99_s"] >= s["latency_p50_s"] > 0


@pytest.mark.parametrize("lanes", [1, 2])
def test_server_admits_at_most_its_batch_tables_of_members(lanes):
    """A budget that would hold every request still admits at most the
    batches' slot count at once; the rest wait for a slot and all complete."""
    from paper_2102_02655_amd import lbprint as LB
    from paper_2102_02655_amd import serving as S

    cap = lanes * LB.Batch.MAX_MEMBERS
    reqs = S.make_requests(count=cap + 6, seed=5, rate=1e6, lmin=16, lmax=18, steps=6)
    budget = sum(LB.footprint(r.cfg) for r in reqs)
    stats = S.Server(budget, chunk=3, lanes=lanes).run(reqs)
    assert sorted(r.id for r in stats.results) == list(range(cap + 6))
    most = max(LB.footprint(r.cfg) for r in reqs)
    assert stats.peak_bytes <= cap * most
