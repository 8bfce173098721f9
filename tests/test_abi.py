"""The C ABI library builds, loads and exports every entry point that
include/lbprint.h declares; host-side validation and sizing work without a
GPU (no kernel is launched here)."""
import ctypes as C
import os
import re

import pytest

from paper_2102_02655_amd import lbprint as LB
from paper_2102_02655_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LB.LIB_PATH):
        from paper_2102_02655_amd import build

        build.build()
    return LB.lib()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lbprint.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lb_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert set(names) == set(LB.EXPORTS)
    for name in names:
        assert hasattr(lib, name), name


def test_struct_sizes_match_header(lib):
    # lb_params: 4 ints, 2x2 doubles ... checked through the library's own
    # validation: a well-formed struct is accepted, a zero box rejected
    cfg = W.static_droplet(n=8, radius=2.0)[0]
    assert LB.footprint(cfg) > 0
    bad = dict(cfg, shape=(0, 8, 8))
    with pytest.raises(LB.LBError) as e:
        LB.footprint(bad)
    assert e.value.status == LB.LB_EINVAL


def test_footprint_scales_with_storage(lib):
    c64 = W.static_droplet(n=32, storage="f64")[0]
    c32 = dict(c64, storage="f32")
    b64, b32 = LB.footprint(c64), LB.footprint(c32)
    N = 32 ** 3
    # two population copies of 38 values dominate
    assert b64 > 2 * 38 * N * 8 and b32 > 2 * 38 * N * 4
    assert 1.9 < b64 / b32 < 2.1
    big = W.print_bed()
    assert LB.footprint(big) < 8 * 2 ** 30  # 512x256x128 FP32 fits comfortably in 288 GB


@pytest.mark.parametrize("change,msg", [
    (dict(tau_b=0.5), "tau_b"),
    (dict(face_zlo="wall", face_zhi="periodic"), "z faces"),
    (dict(rheology="power_law", K=0.0), "power law"),
    (dict(rheology="power_law", K=1e-3, n=1.5), "power law"),
    (dict(tau_min=0.5, rheology="power_law", K=1e-3, n=0.5), "tau_min"),
])
def test_invalid_parameters_rejected(lib, change, msg):
    cfg = W.static_droplet(n=8, radius=2.0)[0]
    cfg.update(change)
    with pytest.raises(LB.LBError) as e:
        LB.footprint(cfg)
    assert e.value.status == LB.LB_EINVAL
    assert msg in str(e.value)


def test_create_rejects_small_or_misaligned_workspace(lib):
    cfg = W.static_droplet(n=8, radius=2.0)[0]
    p = LB.make_params(cfg)
    import numpy as np

    ry = np.ones((8, 8, 8))
    h = C.c_void_p()
    need = LB.footprint(cfg)
    # never dereferenced: the size and alignment checks come first
    rc = lib.lb_create(C.byref(p), ry.ctypes.data, ry.ctypes.data, None, 4096, need - 1, None, C.byref(h))
    assert rc == LB.LB_ENOMEM and not h.value
    rc = lib.lb_create(C.byref(p), ry.ctypes.data, ry.ctypes.data, None, 4097, need, None, C.byref(h))
    assert rc == LB.LB_EINVAL and not h.value
    rc = lib.lb_create(C.byref(p), None, ry.ctypes.data, None, 4096, need, None, C.byref(h))
    assert rc == LB.LB_EINVAL
    assert lib.lb_strerror(LB.LB_ENOMEM) == b"workspace too small"


def test_nozzle_geometry_validation(lib):
    cfg = W.nozzle_extrusion()
    LB.footprint(cfg)
    bad = dict(cfg, nozzle=dict(cfg["nozzle"], tip_z=200.0))
    with pytest.raises(LB.LBError):
        LB.footprint(bad)
    bad = dict(cfg, nozzle=dict(cfg["nozzle"], v=(1.5, 0.0)))
    with pytest.raises(LB.LBError):
        LB.footprint(bad)


def test_step_batch_rejects_bad_arguments_without_touching_the_gpu(lib):
    vp = C.c_void_p
    ks = (C.c_int * 1)(2)
    assert lib.lb_step_batch(None, ks, 1) == LB.LB_EINVAL
    hs = (vp * 1)(None)
    assert lib.lb_step_batch(hs, ks, 1) == LB.LB_EINVAL
    assert lib.lb_step_batch(hs, ks, 0) == LB.LB_EINVAL
    assert b"lb_step_batch" in lib.lb_last_error(None)


def test_unknown_storage_code_rejected(lib):
    cfg = W.static_droplet(n=8, radius=2.0)[0]
    p = LB.make_params(cfg)
    p.storage = 9
    n = C.c_size_t()
    assert lib.lb_footprint(C.byref(p), C.byref(n)) == LB.LB_EINVAL
    assert b"storage" in lib.lb_last_error(None)


def test_reduced_storage_footprint():
    """16-bit deviations (76 B) plus FP32 moments (20 B) per cell and copy,
    against 152 B per cell and copy for FP32 populations."""
    c32 = W.print_bed(storage="f32")
    n = 512 * 256 * 128
    for st in ("bf16dev", "f16dev"):
        b = LB.footprint(dict(c32, storage=st))
        assert b < LB.footprint(c32)
        assert b > 2 * (76 + 20) * n


def test_batch_arguments_rejected_without_the_gpu(lib):
    import ctypes as C

    n = C.c_size_t()
    assert lib.lb_batch_footprint(C.byref(n)) == LB.LB_OK and n.value > 64 * 500
    out = C.c_void_p()
    assert lib.lb_batch_create(1, None, n.value, None, C.byref(out)) == LB.LB_EINVAL
    assert lib.lb_batch_create(9, 256, n.value, None, C.byref(out)) == LB.LB_EINVAL   # unknown storage form
    assert lib.lb_batch_create(1, 257, n.value, None, C.byref(out)) == LB.LB_EINVAL   # misaligned workspace
    assert lib.lb_batch_create(1, 256, 16, None, C.byref(out)) == LB.LB_ENOMEM        # workspace too small
    assert out.value is None
    assert lib.lb_batch_step(None, None, None, 0) == LB.LB_EINVAL
    assert lib.lb_batch_destroy(None) == LB.LB_EINVAL


def test_d2q9_validation_and_footprint(lib):
    """D2Q9 handles live in the x-z plane (ny = 1) with FP64 or FP32
    storage; their population sets are 2 x 9 planes."""
    cfg = W.base_params((64, 1, 32), lattice=9, alpha=(4 / 9, 4 / 9), storage="f32")
    b32 = LB.footprint(cfg)
    N = 64 * 32
    assert 2 * 18 * N * 4 < b32 < LB.footprint(dict(cfg, lattice=19))
    for change, msg in [(dict(shape=(64, 2, 32)), "ny must be 1"),
                        (dict(storage="bf16dev"), "LB_F64 or LB_F32"),
                        (dict(body_g=(0.0, 1e-6, 0.0)), "y components"),
                        (dict(lattice=15), "lattice must be")]:
        bad = dict(cfg, **change)
        if change.get("lattice") == 15:
            p = LB.make_params(dict(cfg))
            p.lattice = 15
            n = C.c_size_t()
            assert lib.lb_footprint(C.byref(p), C.byref(n)) == LB.LB_EINVAL
            continue
        with pytest.raises(LB.LBError) as e:
            LB.footprint(bad)
        assert e.value.status == LB.LB_EINVAL and msg in str(e.value)
