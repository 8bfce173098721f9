"""Pins of the oracle's printing observables (Sec. IV) on hand-built fields
whose thread area, height, width, coverage and pressure are known in closed
form; the pressure is checked against the D2Q9 partial pressure the paper
prints with Eq. (cgoef), p^k = (3/5) rho^k (1 - alpha_k)."""
import numpy as np
import pytest

from oracle import observe as OB

NX, NZ = 40, 20


def cfg(gamma=1.0):
    ab = 4.0 / 9.0
    return dict(lattice=9, alpha=(1.0 - (1.0 - ab) / gamma, ab), rho0=(gamma, 1.0))


def air(c):
    ry = np.zeros((NZ, 1, NX))
    rb = np.full((NZ, 1, NX), c["rho0"][1])
    return ry, rb


def put_ink(c, ry, rb, z, x):
    ry[z, 0, x] = c["rho0"][0]
    rb[z, 0, x] = 0.0


def nosolid():
    return np.zeros((NZ, 1, NX), dtype=bool)


def test_rectangle_thread_has_full_coverage():
    c = cfg()
    ry, rb = air(c)
    for z in range(3):
        for x in range(10, 17):
            put_ink(c, ry, rb, z, x)
    o = OB.observables(c, ry, rb, nosolid(), x_lo=5, x_len=20, z_hi=8)
    assert (o["ink_area"], o["height"], o["width"], o["coverage"]) == (21.0, 3.0, 7.0, 1.0)
    assert o["substrate_ink"] == 7.0


def test_staircase_thread_coverage():
    """Columns of heights w, w-1, ..., 1: A_i = w (w + 1) / 2, A_r = w^2."""
    c = cfg()
    ry, rb = air(c)
    w = 6
    for j in range(w):
        for z in range(w - j):
            put_ink(c, ry, rb, z, 20 + j)
    o = OB.observables(c, ry, rb, nosolid(), x_lo=0, x_len=NX, z_hi=NZ)
    assert o["ink_area"] == w * (w + 1) / 2 and o["height"] == w and o["width"] == w
    assert o["coverage"] == pytest.approx((w + 1) / (2 * w), abs=1e-15)


def test_window_wraps_and_excludes_what_lies_outside():
    c = cfg()
    ry, rb = air(c)
    for x in (NX - 2, NX - 1, 0, 1):  # a thread across the periodic seam
        put_ink(c, ry, rb, 0, x)
    put_ink(c, ry, rb, 0, 10)          # outside the window
    put_ink(c, ry, rb, 9, NX - 1)      # above z_hi (still in the nozzle)
    o = OB.observables(c, ry, rb, nosolid(), x_lo=NX - 3, x_len=6, z_hi=9)
    assert (o["ink_area"], o["height"], o["width"]) == (4.0, 1.0, 4.0)
    # a negative start is the same window
    assert OB.observables(c, ry, rb, nosolid(), x_lo=-3, x_len=6, z_hi=9) == o
    solid = nosolid()
    solid[0, 0, 0] = True              # a head cell is never ink
    o2 = OB.observables(c, ry, rb, solid, x_lo=NX - 3, x_len=6, z_hi=9)
    assert o2["ink_area"] == 3.0 and o2["width"] == 4.0


def test_phase_field_threshold_at_density_ratio_10():
    c = cfg(10.0)
    ry, rb = air(c)
    ry[0, 0, 3], rb[0, 0, 3] = 5.5, 0.5   # rho^N > 0
    ry[0, 0, 4], rb[0, 0, 4] = 4.5, 0.5   # rho^N < 0
    ry[0, 0, 5], rb[0, 0, 5] = 5.0, 0.5   # rho^N = 0: not ink
    o = OB.observables(c, ry, rb, nosolid(), x_lo=0, x_len=NX, z_hi=NZ)
    assert o["ink_area"] == 1.0 and o["width"] == 1.0


@pytest.mark.parametrize("gamma", [1.0, 10.0])
def test_pressure_variation_is_eq_cgoef(gamma):
    c = cfg(gamma)
    ry, rb = air(c)
    ay, ab = c["alpha"]
    put_ink(c, ry, rb, 2, 7)
    ry[3, 0, 7], rb[3, 0, 7] = 1.02 * gamma, 0.01   # the densest ink cell
    o = OB.observables(c, ry, rb, nosolid(), x_lo=0, x_len=NX, z_hi=NZ)
    p0 = 0.6 * 1.0 * (1.0 - ab)
    want = 0.6 * 1.02 * gamma * (1.0 - ay) + 0.6 * 0.01 * (1.0 - ab) - p0
    assert o["p0"] == pytest.approx(p0, rel=1e-14)
    assert o["dp_max"] == pytest.approx(want, rel=1e-12, abs=1e-15)


def test_no_ink_gives_zeros():
    c = cfg()
    ry, rb = air(c)
    o = OB.observables(c, ry, rb, nosolid(), x_lo=0, x_len=NX, z_hi=NZ)
    assert o["ink_area"] == o["height"] == o["width"] == o["coverage"] == o["dp_max"] == 0.0


def test_poi_normalisation():
    v = [OB.poi(1.0, 60, 30, 0.1), OB.poi(0.5, 60, 30, 0.1), OB.poi(1.0, 60, 60, 0.2)]
    assert v[0] == pytest.approx(20.0) and v[1] == pytest.approx(10.0) and v[2] == pytest.approx(5.0)
    n = OB.normalised_poi(v)
    assert n.max() == 1.0 and n[1] == pytest.approx(0.5)
