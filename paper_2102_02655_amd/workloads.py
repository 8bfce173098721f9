"""Seeded synthetic workloads: parameter dicts and initial fields.

This module is shared by the GPU binding's callers and by the oracle's
callers.  It holds no arithmetic of the lattice Boltzmann method itself: only
the physical set-up (box, head, rheology parameters, initial densities) and
seeded random draws.

Parameter dicts use the paper's notation (arXiv:2102.02655):
  shape (nx, ny, nz); alpha (phi_0 of ink Y and air B); rho0 (pure-phase
  densities); A, beta (perturbation and recolouring, Sec. II.A); tau_b (air);
  rheology "newtonian" | "power_law" | "cross" with tau_y / K, n / nu0, nu_inf,
  lambda, m; tau_min, tau_max; zeta_wall, zeta_noz (Eq. (wet)); drag_gamma,
  drag_range, body_g; face_zlo / face_zhi ("periodic" | "wall" | "pressure"),
  u_zlo, u_zhi, rho_zlo, rho_zhi; nozzle = {x0, v, r_in, wall, tip_z, u_ink,
  lid_rho_y} (Sec. II.B).

The paper's own runs are 2-D D2Q9 at density ratio 842 (Sec. III):
printing_2d() is that set-up in the x-z plane (Table I's Cross inks, the
density ratio a parameter); the other printing workloads are the 3-D D3Q19
set-ups at density ratio 1 with a power-law ink, as stated for each.
"""
from __future__ import annotations

import numpy as np

CS2 = 1.0 / 3.0


def base_params(shape, **kw) -> dict:
    """Defaults shared by every workload: alpha = 1/3 for both colours
    (phi_i = w_i on D3Q19, density ratio 1), A = 0.05, beta = 0.7, neutral
    wetting (zeta = 1, a 90 degree contact angle), no drag, no body force."""
    p = dict(
        lattice=19,
        shape=tuple(int(v) for v in shape),
        alpha=(1.0 / 3.0, 1.0 / 3.0),
        rho0=(1.0, 1.0),
        A=0.05,
        beta=0.7,
        eps_g=1e-6,
        tau_b=1.0,
        rheology="newtonian",
        tau_y=1.0,
        K=0.0,
        n=1.0,
        nu0=0.0,
        nu_inf=0.0,
        tau_min=0.51,
        tau_max=2.0,
        rho_eps=1e-6,
        zeta_wall=(1.0, 1.0),
        zeta_noz=(1.0, 1.0),
        drag_gamma=0.0,
        drag_range=4.0,
        body_g=(0.0, 0.0, 0.0),
        face_zlo="periodic",
        face_zhi="periodic",
        u_zlo=(0.0, 0.0, 0.0),
        u_zhi=(0.0, 0.0, 0.0),
        rho_zlo=(0.0, 1.0),
        rho_zhi=(0.0, 1.0),
        nozzle=None,
        storage="f32",
    )
    p.update(kw)
    return p


def ratio10_K(tau_b: float, n: float, gdot_c: float) -> float:
    """Power-law consistency K such that the ink is ten times as viscous as
    the air at the characteristic shear rate gdot_c = |u_ink| / r_in."""
    nu_b = CS2 * (tau_b - 0.5)
    return 10.0 * nu_b * gdot_c ** (1.0 - n)


# ----------------------------------------------------------------- set-ups

def static_droplet(n: int = 32, radius: float = 8.0, seed: int = 2102, trace: float = 0.02,
                   noise: float = 1e-3, storage: str = "f64", tau: float = 1.0):
    """Static droplet: a periodic n^3 box, a sphere of ink (rho_Y = 1, air
    trace) centred at ((n-1)/2,)*3 in air (rho_B = 1, ink trace), Newtonian
    tau for both colours, independent U(-noise, noise) added to rho_Y then
    rho_B, drawn in C order (z, y, x) from default_rng(seed)."""
    cfg = base_params((n, n, n), tau_b=tau, tau_y=tau, storage=storage)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    c = (n - 1) / 2.0
    inside = (x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2 <= radius ** 2
    ry = np.where(inside, 1.0, trace)
    rb = np.where(inside, trace, 1.0)
    rng = np.random.default_rng(seed)
    ry = ry + rng.uniform(-noise, noise, size=ry.shape)
    rb = rb + rng.uniform(-noise, noise, size=rb.shape)
    return cfg, ry, rb


def nozzle_fields(cfg: dict):
    """Initial state of a printing set-up: the nozzle bore (r < r_in, z >= tip)
    holds pure ink, everything else pure air; u = 0."""
    nx, ny, nz = cfg["shape"]
    ry = np.zeros((nz, ny, nx))
    rb = np.ones((nz, ny, nx)) * cfg["rho0"][1]
    noz = cfg.get("nozzle")
    if noz:
        z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        dx = x - noz["x0"][0]
        dy = y - noz["x0"][1]
        dx = dx - nx * np.round(dx / nx)
        dy = dy - ny * np.round(dy / ny)
        bore = (dx ** 2 + dy ** 2 < noz["r_in"] ** 2) & (z >= noz["tip_z"])
        ry = np.where(bore, cfg["rho0"][0], 0.0)
        rb = np.where(bore, 0.0, cfg["rho0"][1])
    return ry, rb


def printing(shape, head_x0, r_in: float, tip_z: float, head_v=(0.0, 0.0), u_ink: float = 0.01,
             n: float = 0.5, sub_u=(0.0, 0.0, 0.0), storage: str = "f32", tau_b: float = 0.53,
             wall: float = 2.0):
    """A printing set-up (3-D reading of the paper's Fig. 1 layout): x, y
    periodic; z = 0 substrate wall (moving at sub_u); top face: inlet lid over
    the bore, constant-air-density face elsewhere; a cylindrical nozzle shell
    (r_in, wall) from tip_z through the top, moving at head_v; power-law ink
    whose viscosity is ten times the air's at gdot_c = u_ink / r_in, tau in
    [0.51, 2.0]; air tau_b = 0.53."""
    K = ratio10_K(tau_b, n, u_ink / r_in)
    cfg = base_params(
        shape,
        tau_b=tau_b,
        rheology="power_law",
        K=K,
        n=n,
        tau_min=0.51,
        tau_max=2.0,
        face_zlo="wall",
        face_zhi="pressure",
        u_zlo=tuple(sub_u),
        rho_zhi=(0.0, 1.0),
        nozzle=dict(x0=tuple(head_x0), v=tuple(head_v), r_in=float(r_in), wall=float(wall), tip_z=float(tip_z),
                    u_ink=(0.0, 0.0, -u_ink), lid_rho_y=1.0),
        storage=storage,
    )
    return cfg


def nozzle_extrusion(storage: str = "f32", shape=(128, 64, 64)):
    """Nozzle extrusion onto a moving substrate: 128x64x64, a fixed nozzle of
    radius 6 (axis at (32, 32), tip z = 12) injecting ink at 0.01, substrate
    moving at 0.005 along x, n = 0.5."""
    return printing(shape, head_x0=(32.0, 32.0), r_in=6.0, tip_z=12.0, head_v=(0.0, 0.0), u_ink=0.01, n=0.5,
                    sub_u=(0.005, 0.0, 0.0), storage=storage)


def print_bed(n: float = 0.5, storage: str = "f32", crop: bool = False):
    """Print-bed filament: 512x256x128 (16.8M cells), head radius 8 (tip z = 16)
    moving along x at 0.01 from (64, 128), ink at 0.01, static substrate.
    crop=True gives the 128x64x32 version with the head from (32, 32)."""
    if crop:
        return printing((128, 64, 32), head_x0=(32.0, 32.0), r_in=8.0, tip_z=16.0, head_v=(0.01, 0.0),
                        u_ink=0.01, n=n, storage=storage)
    return printing((512, 256, 128), head_x0=(64.0, 128.0), r_in=8.0, tip_z=16.0, head_v=(0.01, 0.0),
                    u_ink=0.01, n=n, storage=storage)


def largest_domain(storage: str = "bf16dev"):
    """Largest single domain: 1024x512x384 (201M cells), head radius 24
    (tip z = 48) moving at 0.01 from (256, 256), ink 0.01, n = 0.5."""
    return printing((1024, 512, 384), head_x0=(256.0, 256.0), r_in=24.0, tip_z=48.0, head_v=(0.01, 0.0),
                    u_ink=0.01, n=0.5, storage=storage)


def serving_trace(count: int = 256, seed: int = 4, rate: float = 4.0, lmin: int = 32, lmax: int = 160,
                  steps: int = 2000, storage: str = "f32"):
    """Parameter-sweep requests: Poisson arrivals (mean rate/s), cubic boxes with
    edge L ~ U{lmin..lmax}, ink n ~ U(0.3, 0.9), extrusion u ~ U(0.005, 0.02),
    head u ~ U(0, 0.01); r_in = max(4, round(L/10)), tip 2 r_in, head from
    (L/4, L/2).  Draws from default_rng(seed) in the order arrival, L, n,
    u_ext, u_head."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=count))
    L = rng.integers(lmin, lmax + 1, size=count)
    nn = rng.uniform(0.3, 0.9, size=count)
    uext = rng.uniform(0.005, 0.02, size=count)
    uhead = rng.uniform(0.0, 0.01, size=count)
    reqs = []
    for i in range(count):
        l = int(L[i])
        r_in = float(max(4, int(round(l / 10))))
        cfg = printing((l, l, l), head_x0=(l / 4.0, l / 2.0), r_in=r_in, tip_z=2.0 * r_in,
                       head_v=(float(uhead[i]), 0.0), u_ink=float(uext[i]), n=float(nn[i]), storage=storage)
        reqs.append(dict(id=i, arrival=float(arrivals[i]), cfg=cfg, steps=steps))
    return reqs


def poiseuille(H: int = 32, g: float = 1e-6, tau: float = 1.0, storage: str = "f64"):
    """Body-force-driven channel between static z walls (ink only), periodic
    x, y, one column wide."""
    cfg = base_params((1, 1, H), tau_b=tau, tau_y=tau, face_zlo="wall", face_zhi="wall", body_g=(g, 0.0, 0.0),
                      storage=storage)
    ry = np.ones((H, 1, 1))
    rb = np.zeros((H, 1, 1))
    return cfg, ry, rb


def lattice_units_from_table(nu_mks: float, nu_air_mks: float, tau_air: float, d_mks: float = 0.2e-3,
                             d_lb: float = 60.0):
    """Sec. III unit conversion: dx = d_mks / d_lb, dt = dx^2 nu_air_lb /
    nu_air_mks with nu_air_lb = c_s^2 (tau_air - 1/2); returns (dx, dt, nu_lb)."""
    dx = d_mks / d_lb
    nu_air_lb = CS2 * (tau_air - 0.5)
    dt = dx * dx * nu_air_lb / nu_air_mks
    return dx, dt, nu_mks * dt / (dx * dx)


# ------------------------------------------------------------ 2-D (D2Q9)

# Sec. III, Table I, lattice-unit rows: the Cross law's nu0, nu_inf, lambda
# and exponent for the four alginate inks, and the air's kinematic viscosity
# of each case (tau_B = 0.54, 0.53, 0.52, 0.52).  The printed LB lambda
# exponent (10^-5) is garbled; lambda_MKS / dt gives 10^+5, used here.
TABLE1_LB = {
    "1%-25C": dict(nu0=0.134, nu_inf=0.0181, lam=3.310e5, m=0.751, tau_b=0.54),
    "2%-25C": dict(nu0=0.430, nu_inf=0.0045, lam=8.325e5, m=0.713, tau_b=0.53),
    "3%-25C": dict(nu0=1.991, nu_inf=0.0156, lam=131.0e5, m=0.573, tau_b=0.52),
    "3%-40C": dict(nu0=0.802, nu_inf=0.0221, lam=21.37e5, m=0.737, tau_b=0.52),
}
NU_AIR_MKS = 1.552e-5
D_MKS = 0.2e-3


def ink_speed_lb(case: str, psi: float = 14e-6, rho_ink: float = 1000.0, d_lb: float = 60.0) -> float:
    """Eq. (fluidconv): v_ink = psi / (rho pi (d/2)^2) (psi = 14 mg/s, a
    water-like ink density, d = 0.2 mm), in lattice units of the case's
    dx = d / d_lb and dt = dx^2 nu_air_LB / nu_air_MKS (Eqs. (conv1), (visc))."""
    v = psi / (rho_ink * np.pi * (D_MKS / 2.0) ** 2)
    _, dt, _ = lattice_units_from_table(0.0, NU_AIR_MKS, TABLE1_LB[case]["tau_b"], D_MKS, d_lb)
    return v * dt / (D_MKS / d_lb)


def printing_2d(case: str = "1%-25C", v_ratio: float = 1.0, nx: int = 880, nz: int = 240, d: float = 60.0,
                gap: float = 60.0, wall: float = 4.0, gamma: float = 1.0, head_x0: float = None,
                u_ink: float = None, storage: str = "f32"):
    """The paper's 2-D printing set-up (Sec. III, Fig. 1) on D2Q9 in the x-z
    plane: 880 x 240 nodes, x periodic, a no-slip substrate at z = 0, the top
    face at the air density outside the nozzle and the inlet lid over its
    bore; a nozzle channel of width d (walls `wall` nodes thick) from z = gap
    through the top, starting full of ink at 3/4 of the box (the right side)
    and moving towards -x at v_ratio * v_ink; the ink enters at v_ink
    (Eq. (fluidconv), or u_ink) in the head frame.  Ink: Table I's Cross law
    for `case`; density ratio gamma = rho_Y^0 / rho_B^0 = (1 - alpha_B) /
    (1 - alpha_Y) with alpha_B = 4/9 (phi_i^B = w_i); tau in [0.51, 2.0]."""
    c = TABLE1_LB[case]
    v = ink_speed_lb(case) if u_ink is None else float(u_ink)
    alpha_b = 4.0 / 9.0
    alpha_y = 1.0 - (1.0 - alpha_b) / gamma
    x0 = 0.75 * nx if head_x0 is None else float(head_x0)
    return base_params(
        (nx, 1, nz),
        lattice=9,
        alpha=(alpha_y, alpha_b),
        rho0=(float(gamma), 1.0),
        tau_b=c["tau_b"],
        rheology="cross",
        nu0=c["nu0"],
        nu_inf=c["nu_inf"],
        m=c["m"],
        tau_min=0.51,
        tau_max=2.0,
        face_zlo="wall",
        face_zhi="pressure",
        rho_zhi=(0.0, 1.0),
        nozzle=dict(x0=(x0, 0.0), v=(-v_ratio * v, 0.0), r_in=d / 2.0, wall=float(wall), tip_z=float(gap),
                    u_ink=(0.0, 0.0, -v), lid_rho_y=float(gamma)),
        storage=storage,
        **{"lambda": c["lam"]},
    )


def droplet_2d(n: int = 48, radius: float = 12.0, seed: int = 2102, trace: float = 0.02, noise: float = 1e-3,
               storage: str = "f64", tau: float = 1.0):
    """Static 2-D droplet on D2Q9: a periodic n x 1 x n box, a disc of ink
    (rho_Y = 1, air trace) centred at ((n-1)/2, (n-1)/2) in air, Newtonian tau
    for both colours, independent U(-noise, noise) added to rho_Y then rho_B
    in C order from default_rng(seed); alpha = 4/9 (phi_i = w_i)."""
    cfg = base_params((n, 1, n), lattice=9, alpha=(4.0 / 9.0, 4.0 / 9.0), tau_b=tau, tau_y=tau, storage=storage)
    z, x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    c = (n - 1) / 2.0
    inside = ((x - c) ** 2 + (z - c) ** 2 <= radius ** 2)[:, None, :]
    ry = np.where(inside, 1.0, trace)
    rb = np.where(inside, trace, 1.0)
    rng = np.random.default_rng(seed)
    ry = ry + rng.uniform(-noise, noise, size=ry.shape)
    rb = rb + rng.uniform(-noise, noise, size=rb.shape)
    return cfg, ry, rb
