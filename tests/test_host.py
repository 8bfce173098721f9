"""Host-side logic that needs no GPU: the workspace footprint's population
padding, the benchmark's single-GPU guard and the algebra of the reduced
storage forms' equilibrium."""
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


def test_reduced_storage_equilibrium_affine_form():
    """The reduced storage forms evaluate the D3Q19 equilibrium of a link as
    (w_i / w_1)(t q_i + a) with q_i = 3 c_i.u + 9/2 (c_i.u)^2 and per-cell
    coefficients t_rho = w_1 rho, t_Y = w_1 rho_Y,
    a_T = phi_1^Y rho_Y + phi_1^B rho_B - w_1 (rho_ref + rho k),
    a_Y = rho_Y (phi_1^Y - w_1 k), k = 3/2 u.u, and the rest link as
    Y_0 = g_Y t_Y + (w_0 / w_1) a_Y, T_0 = (g_Y - g_B) t_Y + g_B t_rho + (w_0 / w_1) a_T,
    g_k = (alpha_k - w_0 phi_1^k / w_1) / w_1.  Against the direct definition
    (Sec. II.A: f^{k,eq} = rho_k (phi_i^k + w_i (3 c.u + 9/2 (c.u)^2 - 3/2 u.u)),
    phi_i^k = alpha_k at rest and (1 - alpha_k) w_i / (1 - w_0) otherwise),
    in the stored bases T = f^eq - w_i rho_ref and Y = f^{Y,eq}."""
    import numpy as np

    rng = np.random.default_rng(7)
    w = {0: 1 / 3, 1: 1 / 18, 2: 1 / 36}
    links = [(0, 0, 0)]
    for a in range(3):
        for sg in (1, -1):
            c = [0, 0, 0]
            c[a] = sg
            links.append(tuple(c))
    for a, b in ((0, 1), (0, 2), (1, 2)):
        for sa in (1, -1):
            for sb in (1, -1):
                c = [0, 0, 0]
                c[a], c[b] = sa, sb
                links.append(tuple(c))
    assert len(links) == 19
    for _ in range(300):
        alpha = rng.uniform(0.01, 0.99, 2)
        rho_ref = rng.uniform(0.1, 3.0)
        rY, rB = rng.uniform(0.0, 3.0, 2)
        u = rng.uniform(-0.2, 0.2, 3)
        phi = [[a if s == 0 else (1 - a) * w[s] / (1 - w[0]) for s in range(3)] for a in alpha]
        rho, k, w1 = rY + rB, 1.5 * (u @ u), w[1]
        tr, ty = w1 * rho, w1 * rY
        aT = phi[0][1] * rY + phi[1][1] * rB - w1 * (rho_ref + rho * k)
        aY = rY * (phi[0][1] - w1 * k)
        g = [(alpha[j] - w[0] * phi[j][1] / w1) / w1 for j in range(2)]
        r0 = w[0] / w1
        for c in links:
            s = sum(abs(x) for x in c)
            cu = float(np.dot(c, u))
            E = w[s] * (3 * cu + 4.5 * cu * cu - k)
            Yd = rY * (phi[0][s] + E)
            Td = rY * phi[0][s] + rB * phi[1][s] + rho * E - w[s] * rho_ref
            if s == 0:
                Y = g[0] * ty + r0 * aY
                T = (g[0] - g[1]) * ty + g[1] * tr + r0 * aT
            else:
                q = 3 * cu * (0.5 * 3 * cu + 1)
                Y = w[s] / w1 * (ty * q + aY)
                T = w[s] / w1 * (tr * q + aT)
            assert abs(Y - Yd) <= 1e-13 * (1 + abs(Yd)) and abs(T - Td) <= 1e-13 * (1 + abs(Td)), (c, Y, Yd, T, Td)
