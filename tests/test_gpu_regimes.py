"""GPU (HIP, through the C ABI) against the FP64 oracle in the regimes the
benchmark workloads leave at their defaults:

- the substrate drag -gamma rho_Y (u - u_sub) of Sec. II.B on a moving
  substrate, inside a printing box;
- the Cross law, Eqs. (notnewvisc) and (tauofgammadot), with the 1% alginate
  case of Table I in lattice units (Sec. III);
- the power law in a body-force slit held on both relaxation-time clamps,
  at n = 0.3 and n = 0.9 (the strain-rate solve across its range);
- density ratio 10 (unequal alpha, the phi table of Sec. II.A), in a printing
  box and in a periodic droplet;
- non-neutral wetting (zeta != 1 in Eq. (wet)) on the substrate and nozzle;
- the instability check of lb_step at a check interval.

Tolerances as in test_gpu_parity: relative L2 <= 1e-10 (FP64 storage) and
<= 1e-5 (FP32 storage) on rho_Y, rho_B and u; the FP64 mass ledger's terms
to 1e-9 (FP64) and 1e-4 (FP32) of their size, and the ledger closing on both
sides.
"""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_2102_02655_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-5}
CS2 = 1.0 / 3.0


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def G():
    from paper_2102_02655_amd import lbprint as LB

    LB.lib()
    return LB


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


# FP32 ledger terms are sums of per-link FP32 differences accumulated over
# the run; they follow the state to its FP32 accuracy near each boundary
LEDGER_TOL = {"f64": 1e-9, "f32": 1e-4}


def closure(c, c0):
    """mass(t) - mass(0) - (wall + open + created - deleted), per colour."""
    return c["mass"] - c0["mass"] - (c["mass_wall"] + c["mass_open"] + c["mass_created"] - c["mass_deleted"])


def parity(G, O, cfg, ry, rb, steps, label, u=None, storages=("f64", "f32"), ledger=True, fp32_from=0, tol=None):
    """Run the oracle and the GPU from the same inputs; compare the fields at
    each step count in `steps` (FP32 from step `fp32_from` on) and, with
    `ledger`, the FP64 mass ledger; on both sides the ledger closes."""
    ora = O.OracleSim(dict(cfg, storage="f64"), ry, rb, u=u)
    ref = {0: ora.moments()}
    for t in steps:
        ora.step(t - ora.t)
        ref[t] = ora.moments()
    del ora
    for st in storages:
        sim = G.Sim(dict(cfg, storage=st), ry, rb, u=u)
        c0 = sim.moments()[3]
        for t in steps:
            sim.step(t - sim.t)
            g = sim.moments()
            o = ref[t]
            e = (rel(g[0], o[0]), rel(g[1], o[1]), rel(g[2], o[2]))
            say(f"{label} {st} t={t}: rel-L2 rho_Y {e[0]:.3e} rho_B {e[1]:.3e} u {e[2]:.3e}")
            if st == "f64" or t >= fp32_from:
                bound = (tol or {}).get(st, (TOL[st],) * 3)
                assert all(a <= b for a, b in zip(e, bound)), (label, st, t, e, bound)
            if ledger:
                gc, oc = g[3], o[3]
                for key in ("mass", "mass_wall", "mass_open", "mass_created", "mass_deleted"):
                    scale = max(np.abs(oc[key]).max(), np.abs(oc["mass"]).max() * 1e-6, 1.0)
                    assert np.abs(gc[key] - oc[key]).max() <= LEDGER_TOL[st] * scale, (label, st, key, gc[key],
                                                                                       oc[key])
                m = np.abs(oc["mass"]).sum()
                assert np.abs(closure(oc, ref[0][3])).max() <= 1e-12 * m
                assert np.abs(closure(gc, c0)).max() <= (1e-12 if st == "f64" else 1e-6) * m
        sim.close()
    return ref


def printing_box(**kw):
    cfg = W.printing((40, 32, 24), head_x0=(12.0, 15.5), r_in=4.0, tip_z=10.0, head_v=(0.03, 0.011), u_ink=0.02,
                     n=0.5, sub_u=(0.005, 0.0, 0.0), storage="f64")
    noz = kw.pop("nozzle", None)
    cfg.update(kw)
    if noz:
        cfg["nozzle"].update(noz)
    ry, rb = W.nozzle_fields(cfg)
    return cfg, ry, rb


# ------------------------------------------------------------------- drag

def test_drag_on_moving_substrate(G, O):
    """Printing box over a substrate moving at 0.005 along x with the drag
    switched on in the four layers above it (gamma = 0.05): the ink that
    reaches the substrate is dragged towards the substrate's velocity."""
    cfg, ry, rb = printing_box(drag_gamma=0.05, drag_range=4.0)
    ref = parity(G, O, cfg, ry, rb, (1, 150, 600), "drag")
    # the drag is exercised: ink has reached the drag layers by the end
    assert ref[600][0][:4].max() > 0.1


# ------------------------------------------------------------- Cross law

def test_cross_law_table1_alginate_1pct(G, O):
    """The Cross law with Table I's 1% alginate case at 25 C in lattice units
    (nu0 = 0.134, nu_inf = 0.0181, lambda = 3.31e5, flow index 0.751; air
    tau_B = 0.54, nu_air = 0.0133), clamp [0.51, 2.0]."""
    cfg, ry, rb = printing_box(rheology="cross", nu0=0.134, nu_inf=0.0181, m=0.751, tau_b=0.54)
    cfg["lambda"] = 3.31e5
    parity(G, O, cfg, ry, rb, (1, 150, 600), "cross 1%")


# ---------------------------------------------------------- power-law slit

def _slit_tau(stress, K, n, tmin, tmax):
    """Clamped power-law relaxation time at shear stress `stress` in simple
    shear (the paper's gdot = sqrt 2 du/dz), and du/dz, by bisection."""
    lo, hi = 1e-30, 10.0
    for _ in range(200):
        mid = np.sqrt(lo * hi)
        t = min(max(0.5 + K * (np.sqrt(2) * mid) ** (n - 1) / CS2, tmin), tmax)
        if mid * CS2 * (t - 0.5) > stress:
            hi = mid
        else:
            lo = mid
    m = np.sqrt(lo * hi)
    return min(max(0.5 + K * (np.sqrt(2) * m) ** (n - 1) / CS2, tmin), tmax), m


SLITS = {  # n: (H, K, g, tau_min, tau_max)
    0.3: (24, 1.4678e-4, 2.3714e-6, 0.51, 2.0),
    0.9: (24, 8e-3, 5e-6, 0.5441, 0.5525),
}


@pytest.mark.parametrize("n", sorted(SLITS))
def test_power_law_slit_on_both_clamps(G, O, n):
    """Body-force slit (8 x 4 x H, static walls) started from its steady
    profile: the stress g |z - z_c| puts the wall layers on tau_min and the
    centre layers on tau_max, with the strain-rate solve in between."""
    H, K, g, tmin, tmax = SLITS[n]
    zc = (H - 1) / 2
    taus = [_slit_tau(g * abs(z - zc), K, n, tmin, tmax)[0] for z in range(H)]
    assert taus[0] == tmin and taus[H // 2] == tmax and sum(tmin < t < tmax for t in taus) >= 4
    from scipy.integrate import quad

    prof = np.array([quad(lambda q: _slit_tau(g * q, K, n, tmin, tmax)[1], abs(z - zc), H / 2, limit=200)[0]
                     for z in range(H)])
    nx, ny = 8, 4
    cfg = W.base_params((nx, ny, H), tau_b=0.53, rheology="power_law", K=K, n=n, tau_min=tmin, tau_max=tmax,
                        face_zlo="wall", face_zhi="wall", body_g=(g, 0, 0))
    ry, rb = np.ones((H, ny, nx)), np.zeros((H, ny, nx))
    u = np.zeros((H, ny, nx, 3))
    u[..., 0] = prof[:, None, None]
    parity(G, O, cfg, ry, rb, (1, 100, 400), f"slit n={n}", u=u, ledger=False)


@pytest.mark.parametrize("lattice", [19, 9])
def test_cross_law_slit_spans_the_solve(G, O, lattice):
    """Table I's 1% Cross ink in a body-force slit started from rest: the
    strain rate runs from zero at the centre to its largest at the walls, so
    the relaxation-time solve is exercised across its range, including the
    band (s ~ 1e-6) where a converged iterate once fell out of the bracket.
    FP32 bound on u 5e-4, ten times the 5.0e-5 measured at step 100 (D3Q19;
    1.3e-5 on D2Q9): the ink's non-equilibrium stress is a difference of
    second moments of size rho c_s^2 ~ 0.33 that cancel to ~1e-6 here, so
    FP32 resolves it to a few per cent, and in the Cross law's thinning band
    (lambda gdot ~ 1) the relaxation time follows it."""
    H, g = 24, 1e-6
    ny = 4 if lattice == 19 else 1
    cfg = W.base_params((8, ny, H), lattice=lattice, alpha=((1 / 3, 1 / 3) if lattice == 19 else (4 / 9, 4 / 9)),
                        tau_b=0.54, rheology="cross", nu0=0.134, nu_inf=0.0181, m=0.751, tau_min=0.51, tau_max=2.0,
                        face_zlo="wall", face_zhi="wall", body_g=(g, 0, 0))
    cfg["lambda"] = 3.31e5
    ry, rb = np.ones((H, ny, 8)), np.zeros((H, ny, 8))
    parity(G, O, cfg, ry, rb, (1, 100, 400), f"cross slit D{'3Q19' if lattice == 19 else '2Q9'}", ledger=False,
           fp32_from=100, tol={"f32": (1e-5, 1e-5, 5e-4)})


# ----------------------------------------------------------- density ratio

RATIO = 10.0
ALPHA_10 = (1.0 - (2.0 / 3.0) / RATIO, 1.0 / 3.0)  # gamma = (1 - alpha_B) / (1 - alpha_Y) = 10


def test_density_ratio_10_printing(G, O):
    """Ink ten times as dense as the air (alpha_Y = 0.9333, alpha_B = 1/3,
    rho_Y^0 = 10): unequal phi tables in the equilibria, the anti-bounce-back
    face and the recolouring, with the moving head and the inlet.  Ink and
    head at 0.01 lattice units per step: the ink's sound speed is only
    sqrt((1 - alpha_Y)/2) = 0.18 at this ratio, and at the small box's faster
    speeds (0.02, 0.03) the oracle's own run grows unstable within 900 steps
    and amplifies rounding long before."""
    cfg, ry, rb = printing_box(alpha=ALPHA_10, rho0=(RATIO, 1.0),
                               nozzle=dict(lid_rho_y=RATIO, v=(0.01, 0.005), u_ink=(0.0, 0.0, -0.01)))
    parity(G, O, cfg, ry, rb, (1, 100, 400), "ratio 10 printing")


def test_density_ratio_10_droplet(G, O):
    """A periodic droplet of the dense ink at rest in air (ratio 10)."""
    n = 24
    cfg = W.base_params((n, n, n), alpha=ALPHA_10, rho0=(RATIO, 1.0), tau_b=0.8, tau_y=0.8)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ins = (x - 11.5) ** 2 + (y - 11.5) ** 2 + (z - 11.5) ** 2 <= 36
    rng = np.random.default_rng(10)
    ry = np.where(ins, RATIO, 0.0) + rng.uniform(0, 1e-3, ins.shape)
    rb = np.where(ins, 0.0, 1.0) + rng.uniform(0, 1e-3, ins.shape)
    # FP64 only: a droplet's spurious currents amplify rounding (the FP32
    # droplet at ratio 1 is bounded by the oracle's own noise response in
    # test_gpu_parity); FP32 at this ratio is checked on the printing box
    ref = parity(G, O, cfg, ry, rb, (1, 200, 500), "ratio 10 droplet", storages=("f64",))
    c = ref[500][3]
    assert abs(c["mass"][0] - ry.sum()) < 1e-10 * ry.sum()


# ---------------------------------------------------------------- wetting

def test_non_neutral_wetting(G, O):
    """zeta != 1 in Eq. (wet): a hydrophilic substrate for the ink
    (zeta_wall = (1.25, 0.8)) and a hydrophobic nozzle (zeta_noz = (0.8,
    1.25))."""
    cfg, ry, rb = printing_box(zeta_wall=(1.25, 0.8), zeta_noz=(0.8, 1.25))
    parity(G, O, cfg, ry, rb, (1, 150, 600), "wetting")


# ------------------------------------------------------- instability check

def test_check_interval_reports_instability(G):
    """A body force that accelerates a periodic box past |u| = 0.3: lb_step
    with check_interval 5 stops with LB_EUNSTABLE at the first check past the
    limit, further steps are refused with LB_ESTATE, lb_moments still reads
    the state (and reports LB_EUNSTABLE)."""
    cfg = W.base_params((16, 8, 8), body_g=(0.02, 0.0, 0.0), tau_b=0.9, tau_y=0.9, storage="f32")
    ry, rb = np.full((8, 8, 16), 0.5), np.full((8, 8, 16), 0.5)
    sim = G.Sim(cfg, ry, rb, check_interval=5)
    with pytest.raises(G.LBError) as ei:
        sim.step(100)
    assert ei.value.status == G.LB_EUNSTABLE
    assert sim.t == 15  # u = 0.02 t + 0.01 exceeds 0.3 first at t = 15
    with pytest.raises(G.LBError) as ei:
        sim.step(1)
    assert ei.value.status == G.LB_ESTATE
    ry2, rb2, u, cons = sim.moments(allow_unstable=True)
    assert np.allclose(u[..., 0], 0.02 * 15 + 0.01, rtol=1e-5)
    sim.close()
    # a stable run with the same cadence completes
    cfg["body_g"] = (1e-5, 0.0, 0.0)
    sim = G.Sim(cfg, ry, rb, check_interval=5)
    sim.step(50)
    assert sim.t == 50
    sim.close()
