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
    stats = S.Server(budget, chunk=8, keep_fields=True).run(reqs)
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
