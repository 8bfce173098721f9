"""Write droplet_fp32_noise.json: how much the static-droplet workload
amplifies FP32-sized rounding, measured on the FP64 oracle alone.

The droplet (32^3 periodic, radius 8, trace 0.02, seed 2102, tau = 1) is run
for 1000 steps twice: once clean, once with every population multiplied by
(1 + eps U(-1, 1)) before the first step and after every step (seeded
noise, eps = 2^-24, the relative rounding of an FP32 store; and eps = 2^-20
to show the response is linear in eps).  The relative L2 differences of
rho_Y, rho_B and u between the two runs at t = 1000 are the droplet's
response to rounding of that size.  Only the oracle is called.

Usage: python tests/golden/make_droplet_fp32_noise.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2102_02655_amd import workloads as W  # noqa: E402

STEPS = 1000
SEED = 24


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def noisy_run(cfg, ry, rb, eps):
    rng = np.random.default_rng(SEED)
    s = O.OracleSim(cfg, ry, rb)

    def kick():
        for k in range(2):
            f = s.get_f(k)
            s.set_f(k, f * (1.0 + eps * rng.uniform(-1.0, 1.0, f.shape)))

    kick()
    for _ in range(STEPS):
        s.step(1)
        kick()
    return s.moments()


def main():
    cfg, ry, rb = W.static_droplet()
    clean = O.OracleSim(cfg, ry, rb)
    clean.step(STEPS)
    ref = clean.moments()
    out = {
        "source": "static droplet 32^3 (radius 8, trace 0.02, seed 2102, tau 1, FP64 oracle), "
                  f"{STEPS} steps; populations multiplied by (1 + eps U(-1,1)) before the first step "
                  f"and after every step (numpy default_rng({SEED})); relative L2 against the clean run "
                  "on rho_Y, rho_B, u.  Written by tests/golden/make_droplet_fp32_noise.py (oracle only).",
        "steps": STEPS,
        "response": {},
    }
    for label, eps in (("2^-24", 2.0 ** -24), ("2^-20", 2.0 ** -20)):
        g = noisy_run(cfg, ry, rb, eps)
        out["response"][label] = {"eps": eps, "rel_l2": [rel(g[q], ref[q]) for q in range(3)]}
        print(label, out["response"][label], flush=True)
    with open(os.path.join(HERE, "droplet_fp32_noise.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
