"""Batched stepping (lb_step_batch): one graph launch advances several
simulations of different sizes and storage forms; every result must be
bit-identical to the same simulation stepped alone with lb_step."""
import numpy as np
import pytest

from paper_2102_02655_amd import workloads as W

pytestmark = pytest.mark.gpu


def small_print(shape, head_x0, r_in, tip_z, head_v, u_ink, n, storage):
    cfg = W.printing(shape, head_x0=head_x0, r_in=r_in, tip_z=tip_z, head_v=head_v, u_ink=u_ink, n=n,
                     sub_u=(0.004, 0.0, 0.0), storage=storage)
    ry, rb = W.nozzle_fields(cfg)
    return cfg, ry, rb


CASES = [
    small_print((40, 32, 24), (12.0, 15.5), 4.0, 10.0, (0.03, 0.011), 0.02, 0.5, "f32"),
    small_print((37, 23, 19), (8.0, 9.0), 3.0, 8.0, (0.02, 0.0), 0.015, 0.7, "f32"),
    small_print((64, 48, 32), (20.0, 24.0), 5.0, 12.0, (0.0, 0.01), 0.01, 0.4, "f64"),
    small_print((48, 40, 28), (16.0, 20.0), 4.0, 10.0, (0.015, 0.005), 0.012, 0.6, "bf16dev"),
]


def fields(sim):
    ry, rb, u, cons = sim.moments(dtype=np.float64)
    return ry, rb, u, cons


def assert_same(a, b, what):
    for x, y, name in zip(a[:3], b[:3], ("rho_Y", "rho_B", "u")):
        assert np.array_equal(x, y), f"{what}: {name} differs (max {np.abs(x - y).max()})"
    for key in ("mass", "mom", "mass_wall", "mass_open", "mass_created", "mass_deleted"):
        assert np.array_equal(a[3][key], b[3][key]), f"{what}: {key}"


def test_batch_equals_alone():
    from paper_2102_02655_amd import lbprint as LB

    steps = [(7, 6, 9, 5), (10, 10, 10, 10), (3, 8, 2, 4)]  # per call, per case: odd counts and first steps
    alone = [LB.Sim(cfg, ry, rb) for cfg, ry, rb in CASES]
    mixed = [LB.Sim(cfg, ry, rb) for cfg, ry, rb in CASES]
    for call in steps:
        for s, k in zip(alone, call):
            s.step(k)
        LB.step_batch(mixed, list(call))
    for i, (a, m) in enumerate(zip(alone, mixed)):
        assert a.t == m.t == sum(c[i] for c in steps)
        assert_same(fields(a), fields(m), f"case {i}")


def test_batch_replays_cached_graphs():
    """The same batch stepped again and again reuses the captured graphs;
    the state keeps matching a simulation stepped alone."""
    from paper_2102_02655_amd import lbprint as LB

    cfg, ry, rb = CASES[0]
    cfg2, ry2, rb2 = CASES[1]
    a = LB.Sim(cfg, ry, rb)
    m1, m2 = LB.Sim(cfg, ry, rb), LB.Sim(cfg2, ry2, rb2)
    a.step(1)
    LB.step_batch([m1, m2], [1, 1])
    for _ in range(6):
        a.step(4)
        LB.step_batch([m1, m2], 4)
    assert_same(fields(a), fields(m1), "replayed")


def test_batch_subset_and_alone_in_a_mix_after_a_member_leaves():
    """A member leaves the batch (destroyed); the rest continue; results still
    match stepping alone."""
    from paper_2102_02655_amd import lbprint as LB

    sims = [LB.Sim(cfg, ry, rb) for cfg, ry, rb in CASES]
    ref = LB.Sim(*CASES[1])
    LB.step_batch(sims, 4)
    ref.step(4)
    sims[0].close()
    LB.step_batch(sims[1:], 6)
    ref.step(6)
    assert_same(fields(ref), fields(sims[1]), "after leave")
