"""GPU (HIP, through the C ABI) against the FP64 CPU oracle, element by element
on the same seeded inputs.

Tolerances: FP64 storage, relative L2 <= 1e-10 on rho_Y, rho_B and u; FP32
storage, relative L2 <= 1e-5 on the same fields after 1000 steps (velocity
relative to the oracle's velocity norm over the fluid cells).  The static
droplet is the exception in FP32: its dynamics amplify rounding, so its
FP32 bound is a fixed multiple of the oracle's own response to FP32-sized
rounding noise (tests/golden/droplet_fp32_noise.json, see
test_droplet_fp32).
"""
import json
import os
import sys

import numpy as np
import pytest

from paper_2102_02655_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-5}


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.fixture(scope="module")
def G():
    from paper_2102_02655_amd import lbprint as LB

    LB.lib()
    return LB


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def compare(gpu_fields, ora_fields, tol, label):
    gy, gb, gu, gc = gpu_fields
    oy, ob, ou, oc = ora_fields
    e = (rel(gy, oy), rel(gb, ob), rel(gu, ou))
    say(f"{label}: rel-L2 rho_Y {e[0]:.3e} rho_B {e[1]:.3e} u {e[2]:.3e}")
    assert e[0] <= tol and e[1] <= tol and e[2] <= tol, (label, e)
    return e


# ----------------------------------------------------------- static droplet

@pytest.fixture(scope="module")
def droplet_oracle(O):
    cfg, ry, rb = W.static_droplet()
    s = O.OracleSim(cfg, ry, rb)
    s.step(500)
    f500 = s.moments()
    s.step(500)
    f1000 = s.moments()
    return cfg, ry, rb, f500, f1000


def test_droplet_fp64(G, droplet_oracle):
    """Static droplet, 32^3 periodic, FP64, 500 steps."""
    cfg, ry, rb, f500, _ = droplet_oracle
    sim = G.Sim(dict(cfg, storage="f64"), ry, rb)
    sim.step(500)
    g = sim.moments()
    compare(g, f500, TOL["f64"], "droplet f64 t=500")
    assert np.allclose(g[3]["mass"], f500[3]["mass"], rtol=1e-12)
    assert np.abs(g[3]["mom"] - f500[3]["mom"]).max() < 1e-11


NOISE = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "droplet_fp32_noise.json")))
# The GPU's FP32 path rounds every population after some tens of FP32
# operations, not once: its per-step perturbation is taken as at most 32
# times the 2^-24 storage rounding, and the droplet's response is linear in
# the perturbation (the stored responses at 2^-24 and 2^-20 differ by 16x).
FP32_ROUNDING_FACTOR = 32.0


def test_droplet_fp32(G, droplet_oracle):
    """Static droplet in FP32 storage, 1000 steps.  Bound: FP32_ROUNDING_FACTOR
    times the oracle's own response to FP32-sized rounding noise injected at
    every step (measured on the oracle alone and stored); never above 1e-3.
    FP64 storage over the same 1000 steps stays at 1e-10."""
    cfg, ry, rb, _, f1000 = droplet_oracle
    s64 = G.Sim(dict(cfg, storage="f64"), ry, rb)
    s64.step(1000)
    compare(s64.moments(), f1000, TOL["f64"], "droplet f64 t=1000")
    resp = NOISE["response"]["2^-24"]["rel_l2"]
    lin = [b / a for a, b in zip(resp, NOISE["response"]["2^-20"]["rel_l2"])]
    assert all(8 < r < 32 for r in lin), lin  # linear response: 16x for 16x the noise
    sim = G.Sim(dict(cfg, storage="f32"), ry, rb)
    sim.step(1000)
    g = sim.moments()
    e32 = compare(g, f1000, 1e-3, "droplet f32 t=1000")
    for name, r, e in zip(("rho_Y", "rho_B", "u"), resp, e32):
        say(f"droplet f32 {name}: {e:.3e} = {e / r:.1f} x the oracle's 2^-24 noise response {r:.3e}")
        assert e <= FP32_ROUNDING_FACTOR * r, (name, e, r)
    # FP64 conservation sums of FP32 populations
    assert np.allclose(g[3]["mass"], f1000[3]["mass"], rtol=1e-6)


# ------------------------------------------------------ printing, small box

def small_printing(storage):
    cfg = W.printing((40, 32, 24), head_x0=(12.0, 15.5), r_in=4.0, tip_z=10.0, head_v=(0.03, 0.011), u_ink=0.02,
                     n=0.5, sub_u=(0.005, 0.0, 0.0), storage=storage)
    ry, rb = W.nozzle_fields(cfg)
    return cfg, ry, rb


@pytest.fixture(scope="module")
def printing_oracle(O):
    cfg, ry, rb = small_printing("f64")
    s = O.OracleSim(cfg, ry, rb)
    out = {}
    for t in (1, 37, 300, 1000):
        s.step(t - s.t)
        out[t] = s.moments()
    return cfg, ry, rb, out


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_printing_small_box(G, printing_oracle, storage):
    """Moving head (creation/deletion every few steps), nozzle inlet, moving
    substrate, pressure top face, power-law ink: fields and the FP64 mass
    ledger against the oracle."""
    cfg, ry, rb, ora = printing_oracle
    sim = G.Sim(dict(cfg, storage=storage), ry, rb)
    checks = (1, 37, 300) if storage == "f64" else (1, 37, 300, 1000)
    for t in checks:
        sim.step(t - sim.t)
        g = sim.moments()
        compare(g, ora[t], TOL[storage], f"printing {storage} t={t}")
        gc, oc = g[3], ora[t][3]
        ledger_tol = 1e-9 if storage == "f64" else 1e-5
        for key in ("mass", "mass_wall", "mass_open", "mass_created", "mass_deleted"):
            scale = max(1.0, np.abs(oc["mass"]).max() * 1e-6)
            assert np.abs(gc[key] - oc[key]).max() <= ledger_tol * max(np.abs(oc[key]).max(), scale), (key, gc[key],
                                                                                                     oc[key])
    assert sim.t == checks[-1]


def window_case(storage):
    cfg = W.printing((96, 40, 20), head_x0=(74.0, 30.5), r_in=3.0, tip_z=7.0, head_v=(0.05, 0.03), u_ink=0.02,
                     n=0.5, storage=storage)
    ry, rb = W.nozzle_fields(cfg)
    return cfg, ry, rb


@pytest.fixture(scope="module")
def window_oracle(O):
    cfg, ry, rb = window_case("f64")
    s = O.OracleSim(cfg, ry, rb)
    out = {}
    for t in (200, 600):
        s.step(t - s.t)
        out[t] = s.moments()
    return out


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_head_crossing_the_compact_window(G, window_oracle, storage):
    """The boundary-only arrays keep the head region's columns modulo a
    window: the smallest power of two dividing the extent of at least
    2 ceil(r_out) + 16 = 26 columns (r_out = 5), 32 of 96 in x and 40 (the
    whole extent) in y.
    A head moving at (0.05, 0.03) for 600 steps from (74, 30.5) crosses the
    x window and the periodic boundaries in x and y, so slots are reused by
    cells 32 columns apart while the head's neighbourhood moves through
    them: fields and the FP64 mass ledger against the oracle.  (A window
    that does not divide the extent would alias cells across the periodic
    boundary.)"""
    cfg, ry, rb = window_case(storage)
    sim = G.Sim(cfg, ry, rb)
    for t in (200, 600):
        sim.step(t - sim.t)
        g, o = sim.moments(), window_oracle[t]
        compare(g, o, TOL[storage], f"window crossing {storage} t={t}")
        ledger_tol = 1e-9 if storage == "f64" else 1e-5
        for key in ("mass", "mass_wall", "mass_open", "mass_created", "mass_deleted"):
            scale = max(1.0, np.abs(o[3]["mass"]).max() * 1e-6)
            assert np.abs(g[3][key] - o[3][key]).max() <= ledger_tol * max(np.abs(o[3][key]).max(), scale), key


# ------------------------------------------------- nozzle extrusion (1000)

@pytest.mark.slow
@pytest.mark.timeout(900)
def test_nozzle_extrusion_fp32_1000_steps(G, O):
    """Nozzle extrusion onto a moving substrate, 128x64x64, FP32, 1000 steps:
    relative L2 <= 1e-5 on rho_Y, rho_B, u."""
    cfg = W.nozzle_extrusion(storage="f32")
    ry, rb = W.nozzle_fields(cfg)
    sim = G.Sim(cfg, ry, rb)
    sim.step(1000)
    g = sim.moments()
    s = O.OracleSim(dict(cfg, storage="f64"), ry, rb)
    for k in range(10):
        s.step(100)
        say(f"oracle nozzle extrusion t={s.t}")
    o = s.moments()
    compare(g, o, TOL["f32"], "nozzle extrusion f32 t=1000")


# --------------------------------------------------------------- edge cases

@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_ragged_box(G, O, storage):
    """A box whose cell count is not a multiple of the block size, odd extents
    (FP32: the odd row length keeps every lane on single stores), z walls
    (ghost layers), 60 steps."""
    shape = (37, 23, 19)
    cfg = W.base_params(shape, tau_b=0.8, tau_y=0.7, face_zlo="wall", face_zhi="pressure", u_zlo=(0.01, 0.0, 0.0),
                        body_g=(1e-6, 0.0, -1e-6), storage=storage)
    rng = np.random.default_rng(5)
    z, y, x = np.meshgrid(np.arange(19), np.arange(23), np.arange(37), indexing="ij")
    inside = (x - 18) ** 2 + (y - 11) ** 2 + (z - 8) ** 2 < 36
    ry = np.where(inside, 1.0, 0.0) + rng.uniform(0, 1e-3, inside.shape)
    rb = np.where(inside, 0.0, 1.0) + rng.uniform(0, 1e-3, inside.shape)
    sim = G.Sim(cfg, ry, rb)
    s = O.OracleSim(dict(cfg, storage="f64"), ry, rb)
    sim.step(60)
    s.step(60)
    compare(sim.moments(), s.moments(), TOL[storage], f"ragged {storage} t=60")


def test_single_column_and_pure_phases(G, O):
    """Degenerate boxes: a 1x1xH column (every x/y link wraps onto itself) and
    a box of pure air (no ink anywhere)."""
    cfg, ry, rb = W.poiseuille(H=16, g=1e-5, tau=0.9, storage="f64")
    sim = G.Sim(cfg, ry, rb)
    s = O.OracleSim(cfg, ry, rb)
    sim.step(200)
    s.step(200)
    compare(sim.moments(), s.moments(), TOL["f64"], "column f64 t=200")
    cfg = W.base_params((16, 8, 8), face_zlo="wall", face_zhi="pressure", storage="f32")
    sim = G.Sim(cfg, np.zeros((8, 8, 16)), np.ones((8, 8, 16)))
    sim.step(50)
    gy, gb, gu, gc = sim.moments()
    assert np.all(gy == 0.0) and np.abs(gb - 1.0).max() < 1e-6 and np.abs(gu).max() < 1e-7


def test_moments_do_not_disturb_the_state(G):
    """lb_moments is read-only: interleaving it with lb_step changes nothing
    (bitwise), and two identical runs agree bitwise."""
    cfg, ry, rb = small_printing("f32")
    a = G.Sim(cfg, ry, rb)
    b = G.Sim(cfg, ry, rb)
    c = G.Sim(cfg, ry, rb)
    for _ in range(6):
        a.step(10)
        a.moments()
    b.step(60)
    c.step(60)
    fa, fb, fc = a.moments(), b.moments(), c.moments()
    for q in range(3):
        assert np.array_equal(fa[q], fb[q]) and np.array_equal(fb[q], fc[q])
    for key in fa[3]:
        assert np.array_equal(fa[3][key], fb[3][key])


# ----------------------------------------------------- full-size print bed

@pytest.mark.slow
@pytest.mark.timeout(900)
def test_print_bed_full_size_first_steps(G, O):
    """The benchmark's configuration (512x256x128, FP32, moving head): three
    steps against the oracle over the whole box, and the FP64 mass ledger.
    The head starts on lattice coordinates, so the cells lying exactly on its
    inner and outer radii change class at the first step: 16 nodes are
    created and 80 deleted, at full size as on the 128x64x32 crop."""
    cfg = W.print_bed(storage="f32")
    ry, rb = W.nozzle_fields(cfg)
    sim = G.Sim(cfg, ry, rb)
    sim.step(3)
    g = sim.moments()
    s = O.OracleSim(dict(cfg, storage="f64"), ry, rb)
    s.step(3)
    o = s.moments()
    compare(g, o, TOL["f32"], "print bed f32 t=3")
    gc, oc = g[3], o[3]
    assert oc["mass_created"].sum() > 0 and oc["mass_deleted"].sum() > 0
    for key in ("mass", "mass_wall", "mass_open", "mass_created", "mass_deleted"):
        for k in range(2):  # per colour: the ink's terms are 1e-3 of the air's
            assert abs(gc[key][k] - oc[key][k]) <= 1e-5 * max(abs(oc[key][k]), 1.0), (key, k, gc[key], oc[key])
    del s
