"""GPU tests of the host-side API around the step (timing record, sums-only read-out)."""
import numpy as np
import pytest

from paper_2102_02655_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_timing_record_counts_steps():
    from paper_2102_02655_amd import lbprint

    cfg = W.printing((40, 32, 24), head_x0=(12.0, 15.5), r_in=4.0, tip_z=10.0, head_v=(0.03, 0.011), u_ink=0.02,
                     n=0.5, storage="f32")
    ry, rb = W.nozzle_fields(cfg)
    sim = lbprint.Sim(cfg, ry, rb)
    sim.step(2)
    sim.timing(True)
    sim.step(3)
    sim.timing(False)
    sim.step(2)  # not recorded
    tm = sim.timing_read()
    assert tm["steps"] == 3
    assert tm["step_ms"] > 0 and tm["prep_ms"] >= 0
    assert sim.timing_read()["steps"] == 0  # reading clears
    _, _, _, cons = sim.moments()
    assert np.isfinite(cons["mass"]).all()
    sim.close()


def test_moments_without_fields_gives_the_same_sums():
    """lb_moments with no field outputs (all three pointers null) still
    returns the conserved sums, equal to those of a full read-out."""
    from paper_2102_02655_amd import lbprint

    cfg = W.printing((40, 32, 24), head_x0=(12.0, 15.5), r_in=4.0, tip_z=10.0, head_v=(0.03, 0.011), u_ink=0.02,
                     n=0.5, storage="bf16dev")
    ry, rb = W.nozzle_fields(cfg)
    sim = lbprint.Sim(cfg, ry, rb)
    sim.step(7)
    c_none = sim.moments_device(None, None, None)
    _, _, _, c_full = sim.moments()
    for key in c_full:
        assert np.array_equal(c_none[key], c_full[key]), key
    sim.close()
