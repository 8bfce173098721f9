"""Host-side logic that needs no GPU: the workspace footprint's population
padding and the benchmark's single-GPU guard."""
import os
import subprocess
import sys

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


def test_footprint_includes_population_plane_padding(lib):
    # 512 x 256 x 128 FP32: 64 MiB planes, spaced by 1 MiB + 256 B; two
    # copies of 38 planes
    big = W.print_bed(storage="f32")
    N = 512 * 256 * 128
    assert LB.footprint(big) >= 2 * 38 * (4 * N + (1 << 20) + 256)
    # a small box: planes spaced by 256 B only
    small = W.printing((32, 32, 32), head_x0=(8.0, 16.0), r_in=4.0, tip_z=8.0, storage="f32")
    n = 32 ** 3
    fp = LB.footprint(small)
    assert fp >= 2 * 38 * (4 * n + 256)
    assert fp < 2 * 38 * (4 * n + (1 << 20))
    # the reduced forms: 19 packed words per plane set, 5 moment planes, both padded
    red = W.print_bed(storage="bf16dev")
    assert LB.footprint(red) >= 2 * 19 * (4 * N + (1 << 20) + 256) + 2 * 5 * (4 * N + (1 << 20) + 256)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_footprint_keeps_boundary_arrays_compact(lib):
    """The boundary-only arrays (moment sets, colour fields, macro fields) of
    a walled D3Q19 box hold the z faces' layers and a window around the head,
    not the whole box: the 1024x512x384 BF16-deviation domain needs little
    more than its population state (2 x (19 words + 5 FP32 moments) per cell,
    padded), the 512x256x128 FP32 print bed little more than its 2 x 38
    planes; a periodic box keeps one slot per cell."""
    big = W.largest_domain("bf16dev")
    N = 1024 * 512 * 384
    state = 2 * 19 * (4 * N + (1 << 20) + 256) + 2 * 5 * (4 * N + (1 << 20) + 256)
    fp = LB.footprint(big)
    assert state <= fp <= 40e9, fp
    assert fp - state < 0.05 * state, (fp, state)
    bed = W.print_bed(storage="f32")
    n = 512 * 256 * 128
    pops = 2 * 38 * (4 * n + (1 << 20) + 256)
    assert LB.footprint(bed) - pops < 0.05 * pops
    # periodic droplet: every cell keeps its slots (no faces, no head)
    cfg, _, _ = W.static_droplet(storage="f32")
    m = 32 ** 3
    assert LB.footprint(cfg) >= 2 * 38 * (4 * m + 256) + m * (16 + 60 + 12 + 40)
