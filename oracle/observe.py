"""Printing observables of Sec. IV, from FP64 fields (numpy).

TEST INFRASTRUCTURE ONLY.  The plain reference of the observables the GPU
library reduces on the device (lb_observe); only the tests, the smoke check
and the CPU-baseline leg of the benchmark may import it.  It shares no code
with the GPU library or its binding.

Definitions (Sec. IV and Fig. 4a; the readings are the build's own where the
paper leaves a choice):
- a cell is ink where the phase field rho^N = (rho_Y/rho_Y^0 - rho_B/rho_B^0)
  / (rho_Y/rho_Y^0 + rho_B/rho_B^0) is positive, i.e. rho_Y rho_B^0 >
  rho_B rho_Y^0; solid cells are never ink;
- the printed thread is the ink in a window of columns (periodic in x) below
  a height z_hi (the nozzle tip plane);
- its area A_i is its cell count, its height h is one more than its highest
  cell's z (the substrate wall lies half a cell below z = 0), its width one
  more than the span of its columns, and the circumscribing rectangle's
  area A_r = h * width (coverage ratio A_i / A_r);
- the pressure is the sum of the partial pressures of Eq. (cgoef), p = sum_k
  p^k(rho_k); p0 that of air at rest, p^B(rho_B^0); the pressure variation
  is the largest p - p0 over the ink cells;
- POI = (A_i / A_r) d / (h dp_max), normalised by its maximum over a set of
  runs (Sec. IV).
"""
from __future__ import annotations

import numpy as np

from . import oracle as O


def observables(cfg: dict, rho_y: np.ndarray, rho_b: np.ndarray, solid: np.ndarray, x_lo: int, x_len: int,
                z_hi: int, y: int = 0) -> dict:
    """Observables of the section y of fields shaped (nz, ny, nx)."""
    lat = int(cfg.get("lattice", O.D3Q19))
    ay, ab = cfg["alpha"]
    r0y, r0b = cfg["rho0"]
    ry = np.asarray(rho_y, dtype=np.float64)[:, y, :]
    rb = np.asarray(rho_b, dtype=np.float64)[:, y, :]
    sol = np.asarray(solid, dtype=bool)[:, y, :]
    nz, nx = ry.shape
    ink = ~sol & (ry * r0b > rb * r0y)
    # partial pressures are linear in the density: p^k(rho) = rho p^k(1)
    py, pb = O.partial_pressure(lat, ay, 1.0), O.partial_pressure(lat, ab, 1.0)
    p = ry * py + rb * pb
    p0 = r0b * pb
    s = (np.arange(nx) - int(x_lo)) % nx
    inside = (s < int(x_len))[None, :] & (np.arange(nz) < int(z_hi))[:, None]
    thread = ink & inside
    out = dict(ink_area=float(thread.sum()), height=0.0, width=0.0, coverage=0.0,
               dp_max=float((p - p0)[ink].max()) if ink.any() else 0.0, p0=float(p0),
               substrate_ink=float(ink[0].sum()))
    if thread.any():
        zs, cols = np.nonzero(thread)
        ss = s[cols]
        out["height"] = float(zs.max() + 1)
        out["width"] = float(ss.max() - ss.min() + 1)
        out["coverage"] = out["ink_area"] / (out["height"] * out["width"])
    return out


def poi(coverage: float, d: float, height: float, dp_max: float) -> float:
    """POI proportional to (A_i / A_r) d / (h dp_max) (Sec. IV)."""
    return coverage * d / (height * dp_max)


def normalised_poi(values) -> np.ndarray:
    """POI_i / max_i POI_i (Sec. IV)."""
    v = np.asarray(values, dtype=np.float64)
    return v / v.max()
