"""Reduced storage (populations kept as 16-bit deviations from the local
equilibrium of their source cell, FP32 arithmetic): error against the FP64
oracle, reported and bounded.

Bounds: the stored deviation is rounded to 2^-9 (BF16) or 2^-11 (FP16 of
delta / w_i) of itself; deviations are about 1e-2 of a population near the
interface and the head, so each step perturbs a population by up to ~2e-5
(BF16) / ~5e-6 (FP16) relative.  Measured over the runs below: rho_Y 2-4e-5,
u 1.5-2.6e-4 (BF16); rho_Y 2-3e-6, u 2-3e-5 (FP16).  The asserted bounds are
ten times the measured values; the FP32 plain form is listed for reference."""
import os

import numpy as np
import pytest

from paper_2102_02655_amd import workloads as W

pytestmark = pytest.mark.gpu

BOUND = {  # (rho_Y, rho_B, u) relative L2 vs the FP64 oracle
    "bf16dev": (4e-4, 6e-5, 3e-3),
    "f16dev": (4e-5, 8e-6, 3e-4),
}


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def small_print_oracle():
    from oracle import oracle as O

    cfg = W.printing((40, 32, 24), head_x0=(12.0, 15.5), r_in=4.0, tip_z=10.0, head_v=(0.03, 0.011), u_ink=0.02,
                     n=0.5, sub_u=(0.005, 0.0, 0.0), storage="f64")
    ry, rb = W.nozzle_fields(cfg)
    o = O.OracleSim(cfg, ry, rb)
    o.step(200)
    return cfg, ry, rb, o.moments()


@pytest.mark.parametrize("storage", ["bf16dev", "f16dev"])
def test_reduced_storage_small_print(small_print_oracle, storage):
    from paper_2102_02655_amd import lbprint as LB

    cfg, ry, rb, ref = small_print_oracle
    s = LB.Sim(dict(cfg, storage=storage), ry, rb)
    s.step(200)
    g = s.moments(dtype=np.float64)
    errs = (rel(g[0], ref[0]), rel(g[1], ref[1]), rel(g[2], ref[2]))
    print(f"{storage} 200 steps: rho_Y {errs[0]:.2e} rho_B {errs[1]:.2e} u {errs[2]:.2e}")
    for e, b in zip(errs, BOUND[storage]):
        assert e <= b, (errs, BOUND[storage])
    # the mass ledger closes to the rounding of the stored deviations
    c0 = LB.Sim(dict(cfg, storage=storage), ry, rb).moments()[3]
    c = g[3]
    for k in range(2):
        lhs = c["mass"][k] - c0["mass"][k]
        rhs = c["mass_wall"][k] + c["mass_open"][k] + c["mass_created"][k] - c["mass_deleted"][k]
        assert abs(lhs - rhs) <= 1e-4 * c["mass"][1], (k, lhs, rhs)
    s.close()


@pytest.mark.slow
@pytest.mark.timeout(900)
@pytest.mark.parametrize("storage", ["bf16dev", "f16dev"])
def test_reduced_storage_nozzle_extrusion_1000_steps(storage):
    """The 128x64x64 extrusion onto the moving substrate, 1000 steps."""
    from oracle import oracle as O
    from paper_2102_02655_amd import lbprint as LB

    cfg = W.nozzle_extrusion(storage="f64")
    ry, rb = W.nozzle_fields(cfg)
    o = O.OracleSim(cfg, ry, rb)
    o.step(1000)
    ref = o.moments()
    s = LB.Sim(dict(cfg, storage=storage), ry, rb)
    s.step(1000)
    g = s.moments(dtype=np.float64)
    errs = (rel(g[0], ref[0]), rel(g[1], ref[1]), rel(g[2], ref[2]))
    print(f"{storage} extrusion 1000 steps: rho_Y {errs[0]:.2e} rho_B {errs[1]:.2e} u {errs[2]:.2e}")
    for e, b in zip(errs, BOUND[storage]):
        assert e <= b, (errs, BOUND[storage])


@pytest.fixture(scope="module")
def print_bed_oracle():
    from oracle import oracle as O

    cfg = W.print_bed(storage="f64")
    ry, rb = W.nozzle_fields(cfg)
    o = O.OracleSim(cfg, ry, rb)
    o.step(3)
    out = o.moments()
    del o
    return cfg, ry, rb, out


@pytest.mark.slow
@pytest.mark.parametrize("storage", ["bf16dev", "f16dev"])
def test_reduced_storage_print_bed_full_size(print_bed_oracle, storage):
    """The 512x256x128 print bed (population and moment planes of 64 MiB,
    spaced by padding): three steps against the oracle over the whole box."""
    from paper_2102_02655_amd import lbprint as LB

    cfg, ry, rb, ref = print_bed_oracle
    s = LB.Sim(dict(cfg, storage=storage), ry, rb)
    s.step(3)
    g = s.moments(dtype=np.float64)
    errs = (rel(g[0], ref[0]), rel(g[1], ref[1]), rel(g[2], ref[2]))
    print(f"{storage} print bed 3 steps: rho_Y {errs[0]:.2e} rho_B {errs[1]:.2e} u {errs[2]:.2e}")
    for e, b in zip(errs, BOUND[storage]):
        assert e <= b, (errs, BOUND[storage])
    s.close()


# Density ratio 10 (alpha_Y = 0.9333, alpha_B = 1/3, rho_Y^0 = 10) on the
# small printing box: only at unequal alpha are the rest link's equilibrium
# coefficients g_k of the reduced forms non-zero.  The stored deviations are
# large next to the slow flow here (ink and head at 0.01), so the errors are
# larger than at ratio 1: measured after 400 steps BF16 3.3e-4 / 1.2e-4 /
# 9.9e-3 and FP16 3.3e-5 / 1.4e-5 / 1.0e-3 (rho_Y / rho_B / u); the bounds
# are ten times those.  The two forms' errors differ by their mantissas
# (2^-8 against 2^-11 relative), as the rounding of the deviations predicts;
# an equilibrium that the encoder and a decoder evaluated differently would
# add an error that does not depend on the storage precision.
RATIO10_BOUND = {"bf16dev": (4e-3, 1.5e-3, 1e-1), "f16dev": (4e-4, 1.5e-4, 1e-2)}


def test_reduced_storage_density_ratio_10():
    from oracle import oracle as O
    from paper_2102_02655_amd import lbprint as LB

    ratio = 10.0
    cfg = W.printing((40, 32, 24), head_x0=(12.0, 15.5), r_in=4.0, tip_z=10.0, head_v=(0.03, 0.011), u_ink=0.02,
                     n=0.5, sub_u=(0.005, 0.0, 0.0), storage="f64")
    cfg.update(alpha=(1.0 - (2.0 / 3.0) / ratio, 1.0 / 3.0), rho0=(ratio, 1.0))
    cfg["nozzle"].update(lid_rho_y=ratio, v=(0.01, 0.005), u_ink=(0.0, 0.0, -0.01))
    ry, rb = W.nozzle_fields(cfg)
    o = O.OracleSim(cfg, ry, rb)
    o.step(400)
    ref = o.moments()
    errs = {}
    for st in ("bf16dev", "f16dev"):
        s = LB.Sim(dict(cfg, storage=st), ry, rb)
        c0 = s.moments()[3]
        s.step(400)
        g = s.moments(dtype=np.float64)
        errs[st] = (rel(g[0], ref[0]), rel(g[1], ref[1]), rel(g[2], ref[2]))
        print(f"ratio 10 {st} 400 steps: rho_Y {errs[st][0]:.2e} rho_B {errs[st][1]:.2e} u {errs[st][2]:.2e}")
        for e, b in zip(errs[st], RATIO10_BOUND[st]):
            assert e <= b, (st, errs[st], RATIO10_BOUND[st])
        c = g[3]
        for k in range(2):
            lhs = c["mass"][k] - c0["mass"][k]
            rhs = c["mass_wall"][k] + c["mass_open"][k] + c["mass_created"][k] - c["mass_deleted"][k]
            assert abs(lhs - rhs) <= 1e-4 * c["mass"][1], (st, k, lhs, rhs)
        s.close()
    assert all(b > 4 * f for b, f in zip(errs["bf16dev"], errs["f16dev"])), errs


# The print-bed crop (128x64x32, same head, speeds and rheology as the full
# box), every storage form against the FP64 oracle.  The default run takes
# n = 0.5 over 1000 steps (about half a minute of oracle time);
# LB_CROP_FULL=1 runs n = 0.3, 0.5 and 0.8 over 5000 steps (the report).
CROP_FULL = bool(os.environ.get("LB_CROP_FULL"))
CROP_N = [0.3, 0.5, 0.8] if CROP_FULL else [0.5]
CROP_STEPS = 5000 if CROP_FULL else 1000
CROP_BOUND = {  # (rho_Y, rho_B, u) relative L2 (errors grow with steps): about ten times
    # the largest measured after 5000 steps over n = 0.3, 0.5, 0.8 (FP32 1.2e-5 / 2.6e-6 / 2.6e-5,
    # BF16 1.0e-4 / 2.1e-5 / 1.9e-4, FP16 1.6e-5 / 3.4e-6 / 3.3e-5)
    "f32": (2e-4, 4e-5, 4e-4),
    "bf16dev": (1e-3, 2e-4, 2e-3),
    "f16dev": (2e-4, 4e-5, 4e-4),
}
if CROP_STEPS == 1000:
    # plain FP32 storage is held to the FP32 bar of 1e-5 after 1000 steps
    CROP_BOUND["f32"] = (1e-5, 1e-5, 1e-5)


@pytest.mark.slow
@pytest.mark.parametrize("n", CROP_N)
def test_storage_forms_print_bed_crop(n):
    from oracle import oracle as O
    from paper_2102_02655_amd import lbprint as LB

    cfg = W.print_bed(n=n, storage="f64", crop=True)
    ry, rb = W.nozzle_fields(cfg)
    o = O.OracleSim(cfg, ry, rb)
    for k in range(CROP_STEPS // 500):
        o.step(500)
        print(f"oracle crop n={n}: {500 * (k + 1)} steps", flush=True)
    ref = o.moments()
    del o
    for st in ("f32", "bf16dev", "f16dev"):
        s = LB.Sim(dict(cfg, storage=st), ry, rb)
        s.step(CROP_STEPS)
        g = s.moments(dtype=np.float64)
        errs = (rel(g[0], ref[0]), rel(g[1], ref[1]), rel(g[2], ref[2]))
        print(f"crop n={n} {st} {CROP_STEPS} steps: rho_Y {errs[0]:.2e} rho_B {errs[1]:.2e} u {errs[2]:.2e}", flush=True)
        s.close()
        for e, b in zip(errs, CROP_BOUND[st]):
            assert e <= b, (st, errs, CROP_BOUND[st])


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_largest_domain_first_steps_against_an_oracle_crop():
    """The 1024x512x384 domain (BF16 deviations, the largest-domain
    benchmark's launch configuration: compact boundary arrays, 39.9 GB)
    against the oracle where it can follow: the state starts as pure air at
    rest outside the ink-filled bore, an exact fixed point of the step away
    from the head, and a step moves a disturbance at most two cells (pull and
    colour stencil).  After three steps the box therefore equals, cell for
    cell, a 128x128x384 crop centred on the head with the same walls, top
    face and nozzle, which the FP64 oracle runs (its disturbance reaches
    31 cells from the axis; beyond, both hold air at rest to rounding).
    Also: the far field is at rest on the GPU, and the FP64 mass ledger
    closes."""
    import torch

    from oracle import oracle as O
    from paper_2102_02655_amd import lbprint as LB

    cfg = W.largest_domain("bf16dev")
    nx, ny, nz = cfg["shape"]
    N = nx * ny * nz
    fp = LB.footprint(cfg)
    assert fp <= 40e9, fp
    ry, rb = W.nozzle_fields(cfg)
    sim = LB.Sim(cfg, ry, rb)
    del ry, rb
    c0 = sim.moments_device(None, None, None)
    sim.step(3)
    dev = torch.device("cuda:0")
    gy = torch.empty((nz, ny, nx), dtype=torch.float32, device=dev)
    gb = torch.empty_like(gy)
    gu = torch.empty((nz, ny, nx, 3), dtype=torch.float32, device=dev)
    c1 = sim.moments_device(gy, gb, gu)
    sim.close()
    # the ledger: mass change = wall + open + created - deleted
    for k in range(2):
        lhs = c1["mass"][k] - c0["mass"][k]
        rhs = c1["mass_wall"][k] + c1["mass_open"][k] + c1["mass_created"][k] - c1["mass_deleted"][k]
        assert abs(lhs - rhs) <= 1e-9 * c1["mass"][1], (k, lhs, rhs)
    # the crop around the head axis at (256, 256)
    x0, y0, w = 256 - 64, 256 - 64, 128
    far = torch.ones((ny, nx), dtype=torch.bool, device=dev)
    far[y0:y0 + w, x0:x0 + w] = False
    assert float((gb[:, far] - 1.0).abs().max()) <= 1e-6 and float(gy[:, far].abs().max()) <= 1e-6
    assert float(gu[:, far].abs().max()) <= 1e-6
    g = (gy[:, y0:y0 + w, x0:x0 + w].double().cpu().numpy(), gb[:, y0:y0 + w, x0:x0 + w].double().cpu().numpy(),
         gu[:, y0:y0 + w, x0:x0 + w].double().cpu().numpy())
    del gy, gb, gu
    crop = W.printing((w, w, nz), head_x0=(64.0, 64.0), r_in=24.0, tip_z=48.0, head_v=(0.01, 0.0), u_ink=0.01,
                      n=0.5, storage="f64")
    cy, cb = W.nozzle_fields(crop)
    o = O.OracleSim(crop, cy, cb)
    o.step(3)
    ref = o.moments()
    # the crop's own edge columns are far field too
    edge = np.ones((w, w), dtype=bool)
    edge[8:w - 8, 8:w - 8] = False
    assert np.abs(ref[1][:, edge] - 1.0).max() <= 1e-12 and np.abs(ref[2][:, edge]).max() <= 1e-12
    errs = (rel(g[0], ref[0]), rel(g[1], ref[1]), rel(g[2], ref[2]))
    print(f"1024x512x384 bf16dev, 3 steps, crop around the head: rho_Y {errs[0]:.2e} rho_B {errs[1]:.2e} "
          f"u {errs[2]:.2e}; footprint {fp / 1e9:.2f} GB, {N} cells")
    for e, b in zip(errs, BOUND["bf16dev"]):
        assert e <= b, (errs, BOUND["bf16dev"])
