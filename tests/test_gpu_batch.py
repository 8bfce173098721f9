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


# --------------------------------------------- batches over a device slot table

def cases_of(storage):
    return [small_print(shape, x0, r, tip, v, ui, n, storage) for shape, x0, r, tip, v, ui, n in (
        ((40, 32, 24), (12.0, 15.5), 4.0, 10.0, (0.03, 0.011), 0.02, 0.5),
        ((37, 23, 19), (8.0, 9.0), 3.0, 8.0, (0.02, 0.0), 0.015, 0.7),
        ((64, 48, 32), (20.0, 24.0), 5.0, 12.0, (0.0, 0.01), 0.01, 0.4),
        ((20, 70, 16), (9.0, 30.0), 3.0, 6.0, (0.0, 0.04), 0.012, 0.6),
    )]


@pytest.mark.parametrize("storage", ["f32", "bf16dev", "f16dev", "f64"])
def test_slot_table_batch_equals_alone(storage):
    """Members of different sizes advance by their own counts per call (odd
    counts, a first step, a member sitting a call out); every field and FP64
    sum equals the member stepped alone, bit for bit."""
    from paper_2102_02655_amd import lbprint as LB

    cases = cases_of(storage)
    calls = [(7, 6, 9, 1), (10, 10, 10, 10), (3, 8, 0, 4), (12, 1, 5, 12)]
    alone = [LB.Sim(cfg, ry, rb) for cfg, ry, rb in cases]
    mixed = [LB.Sim(cfg, ry, rb) for cfg, ry, rb in cases]
    batch = LB.Batch(storage)
    for call in calls:
        for s, k in zip(alone, call):
            s.step(k)
        batch.step(mixed, list(call))
    for i, (a, m) in enumerate(zip(alone, mixed)):
        assert a.t == m.t == sum(c[i] for c in calls)
        assert_same(fields(a), fields(m), f"{storage} member {i}")
    batch.close()


def test_slot_table_membership_changes_and_recapture():
    """Members join, leave and are destroyed between calls; a larger member
    and a longer call outgrow the captured graph (it is captured again); the
    results still equal lone runs."""
    from paper_2102_02655_amd import lbprint as LB

    cases = cases_of("f32")
    big = small_print((96, 64, 40), (30.0, 31.5), 6.0, 14.0, (0.02, 0.0), 0.015, 0.5, "f32")
    alone = {i: LB.Sim(*c) for i, c in enumerate(cases)}
    alone[4] = LB.Sim(*big)
    mixed = {i: LB.Sim(*c) for i, c in enumerate(cases)}
    batch = LB.Batch("f32")
    schedule = [  # (members, steps)
        ([0, 1], 4),
        ([0, 1, 2], 4),
        ([1, 2], 6),        # member 0 leaves
        ([1, 2, 3], 4),
        ([2, 3], 2),        # member 1 leaves and is destroyed
        ([2, 3, 4], 4),     # a larger member joins: more blocks than captured
        ([2, 3, 4], 16),    # a longer call: more steps than captured
        ([3, 4], 6),
    ]
    for members, k in schedule:
        if 4 in members and 4 not in mixed:
            mixed[4] = LB.Sim(*big)
        for i in members:
            alone[i].step(k)
        batch.step([mixed[i] for i in members], k)
        if members == [2, 3]:
            mixed[1].close()
            alone[1].close()
    for i in (0, 2, 3, 4):
        assert alone[i].t == mixed[i].t
        assert_same(fields(alone[i]), fields(mixed[i]), f"member {i}")
    batch.close()


def test_slot_table_members_on_their_own_streams():
    """Members created on their own streams, read out between batch calls
    (on their streams), keep their order with the batch stream."""
    import torch

    from paper_2102_02655_amd import lbprint as LB

    cases = cases_of("bf16dev")[:3]
    alone = [LB.Sim(*c) for c in cases]
    mixed = [LB.Sim(*c, stream=torch.cuda.Stream()) for c in cases]
    batch = LB.Batch("bf16dev")
    for k in (5, 8, 8):
        for s in alone:
            s.step(k)
        batch.step(mixed, k)
        for a, m in zip(alone, mixed):
            assert_same(fields(a), fields(m), f"after {a.t} steps")
    mixed[0].step(3)  # a member stepped on its own between calls
    alone[0].step(3)
    batch.step(mixed, [4, 4, 4])
    for a in alone:
        a.step(4)
    for a, m in zip(alone, mixed):
        assert_same(fields(a), fields(m), "after a lone step in between")
    batch.close()
