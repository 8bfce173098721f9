"""lb_moments_noalloc (the read-out whose per-call partial sums live in the
library's static device array) against lb_moments, through the C ABI: fields
bit for bit, FP64 sums to 1e-12, on two calls in a row with the second on a
smaller simulation, and the state left as it was."""
import ctypes as C

import numpy as np
import pytest

from paper_2102_02655_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def LB():
    from paper_2102_02655_amd import lbprint as L

    L.lib()
    return L


def read(LB, sim, fn, dtype=np.float64, device=False):
    nx, ny, nz = sim.shape
    cons = LB.Conserved()
    code = 0 if np.dtype(dtype) == np.float64 else 1
    if device:
        import torch

        td = torch.float64 if code == 0 else torch.float32
        ry = torch.zeros((nz, ny, nx), dtype=td, device=sim.device)
        rb = torch.zeros_like(ry)
        u = torch.zeros((nz, ny, nx, 3), dtype=td, device=sim.device)
        rc = fn(sim._h, ry.data_ptr(), rb.data_ptr(), u.data_ptr(), 1, code, C.byref(cons))
        out = (ry.cpu().numpy(), rb.cpu().numpy(), u.cpu().numpy())
    else:
        ry = np.zeros((nz, ny, nx), dtype=dtype)
        rb = np.zeros_like(ry)
        u = np.zeros((nz, ny, nx, 3), dtype=dtype)
        rc = fn(sim._h, ry.ctypes.data, rb.ctypes.data, u.ctypes.data, 0, code, C.byref(cons))
        out = (ry, rb, u)
    assert rc == LB.LB_OK, LB.lib().lb_last_error(sim._h)
    return out, cons.as_dict()


def same(LB, sim, label, **kw):
    lib = LB.lib()
    a, ca = read(LB, sim, lib.lb_moments, **kw)
    b, cb = read(LB, sim, lib.lb_moments_noalloc, **kw)
    for q in range(3):
        assert np.array_equal(a[q], b[q]), (label, q)
    for key in ca:
        scale = max(np.abs(ca[key]).max(), 1.0)
        assert np.abs(ca[key] - cb[key]).max() <= 1e-12 * scale, (label, key, ca[key], cb[key])
    print(f"{label}: fields equal, sums {cb['mass']} vs {ca['mass']}", flush=True)


def test_noalloc_readout_matches_lb_moments(LB):
    # 524,288 cells: 2048 blocks' worth, so the fixed grid of 1024 blocks
    # takes two cells per thread
    big = W.printing((128, 64, 64), head_x0=(40.0, 31.5), r_in=6.0, tip_z=12.0, head_v=(0.04, 0.013), u_ink=0.02,
                     n=0.5, sub_u=(0.005, 0.0, 0.0), storage="f32")
    small = W.printing((24, 16, 12), head_x0=(8.0, 7.5), r_in=3.0, tip_z=5.0, head_v=(0.05, 0.0), u_ink=0.02,
                       n=0.5, storage="f64")
    s1 = LB.Sim(big, *W.nozzle_fields(big))
    s1.step(37)
    same(LB, s1, "large f32 host")
    s2 = LB.Sim(small, *W.nozzle_fields(small))
    s2.step(23)
    same(LB, s2, "small f64 host")  # second call, smaller input: stale slots must not leak in
    same(LB, s2, "small f64 device f32", dtype=np.float32, device=True)
    same(LB, s1, "large f32 again")
    # the read-out leaves the state alone: stepping on matches a twin that never read out
    twin = LB.Sim(small, *W.nozzle_fields(small))
    twin.step(23)
    s2.step(10)
    twin.step(10)
    a, ca = read(LB, s2, LB.lib().lb_moments_noalloc)
    b, cb = read(LB, twin, LB.lib().lb_moments)
    for q in range(3):
        assert np.array_equal(a[q], b[q])
    for s in (s1, s2, twin):
        s.close()


def test_noalloc_readout_first_step_and_periodic_box(LB):
    """No pending creation (a periodic box without a head, and a handle
    before its first step): the pending-creation slots are not read."""
    cfg, ry, rb = W.static_droplet(n=16, radius=4.0, storage="f32")
    s = LB.Sim(cfg, ry, rb)
    same(LB, s, "droplet t=0")
    s.step(5)
    same(LB, s, "droplet t=5")
    s.close()
    big = W.print_bed(storage="bf16dev", crop=True)
    s = LB.Sim(big, *W.nozzle_fields(big))
    same(LB, s, "crop bf16 t=0")
    s.step(3)
    same(LB, s, "crop bf16 t=3")
    s.close()
