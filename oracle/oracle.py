"""ctypes binding of the FP64 CPU oracle (``liblbo.so``).

TEST INFRASTRUCTURE ONLY.  The oracle is the slow, literal FP64 reference of
the regularized colour-gradient lattice Boltzmann model of arXiv:2102.02655
(Sec. II.A-B); the GPU library is checked against it.  Only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import this module.
It shares no code with the GPU library or its binding.

Parameters arrive as a plain dict in the paper's notation (see
``paper_2102_02655_amd.workloads``); this module converts it to the oracle's
own C struct.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblbo.so")

D2Q9 = 9
D3Q19 = 19
_RHEO = {"newtonian": 0, "power_law": 1, "cross": 2}
_FACE = {"periodic": 0, "wall": 1, "pressure": 2}

_d2 = C.c_double * 2
_d3 = C.c_double * 3


class _Params(C.Structure):
    _fields_ = [
        ("lattice", C.c_int),
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("alpha", _d2), ("rho0", _d2),
        ("A", C.c_double), ("beta", C.c_double), ("eps_g", C.c_double),
        ("tau_b", C.c_double),
        ("rheology", C.c_int),
        ("tau_y", C.c_double),
        ("K", C.c_double), ("n", C.c_double),
        ("nu0", C.c_double), ("nu_inf", C.c_double), ("lam", C.c_double), ("m", C.c_double),
        ("tau_min", C.c_double), ("tau_max", C.c_double),
        ("rho_eps", C.c_double),
        ("zeta_wall", _d2), ("zeta_noz", _d2),
        ("drag_gamma", C.c_double), ("drag_range", C.c_double),
        ("body_g", _d3),
        ("face_zlo", C.c_int), ("face_zhi", C.c_int),
        ("u_zlo", _d3), ("u_zhi", _d3),
        ("rho_zlo", _d2), ("rho_zhi", _d2),
        ("has_nozzle", C.c_int),
        ("noz_x0", _d2), ("noz_v", _d2),
        ("noz_r_in", C.c_double), ("noz_wall", C.c_double), ("noz_tip_z", C.c_double),
        ("u_ink", _d3),
        ("lid_rho_y", C.c_double),
        ("collide", C.c_int),
    ]


class Conserved(C.Structure):
    _fields_ = [
        ("mass", _d2), ("mom", _d3),
        ("mass_wall", _d2), ("mass_open", _d2),
        ("mass_created", _d2), ("mass_deleted", _d2),
    ]

    def as_dict(self) -> dict:
        return {name: np.array(list(getattr(self, name))) for name, _ in self._fields_}


_lib = None


def lib():
    """Load ``liblbo.so`` (built by ``oracle/build.py``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"oracle library missing: {_LIB_PATH}; run oracle/build.py")
        L = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        L.lbo_lattice.argtypes = [C.c_int, ip, ip, ip, dp, dp]
        L.lbo_phi.argtypes = [C.c_int, C.c_double, dp]
        L.lbo_B.argtypes = [C.c_int, dp]
        L.lbo_partial_pressure.argtypes = [C.c_int, C.c_double, C.c_double]
        L.lbo_partial_pressure.restype = C.c_double
        L.lbo_feq.argtypes = [C.c_int, C.c_double, C.c_double, dp, dp]
        L.lbo_regularize.argtypes = [C.c_int, C.c_double, C.c_double, dp, dp, dp]
        L.lbo_perturbation.argtypes = [C.c_int, C.c_double, dp, dp, dp]
        L.lbo_recolour.argtypes = [C.c_int, dp, C.c_double, C.c_double, C.c_double, C.c_double, dp, dp, dp, dp]
        L.lbo_tau_ink.argtypes = [C.POINTER(_Params), C.c_double, C.c_double, dp, dp]
        L.lbo_wall_density.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int, C.c_int]
        L.lbo_wall_density.restype = C.c_double
        L.lbo_gradient.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, dp, dp]
        L.lbo_create.argtypes = [C.POINTER(_Params), dp, dp, dp, C.POINTER(C.c_void_p)]
        L.lbo_step.argtypes = [C.c_void_p, C.c_int]
        L.lbo_moments.argtypes = [C.c_void_p, dp, dp, dp, C.POINTER(Conserved)]
        L.lbo_get_f.argtypes = [C.c_void_p, C.c_int, dp]
        L.lbo_set_f.argtypes = [C.c_void_p, C.c_int, dp]
        L.lbo_solid.argtypes = [C.c_void_p, C.POINTER(C.c_uint8)]
        L.lbo_velocity_index.argtypes = [C.c_void_p, ip]
        L.lbo_time.argtypes = [C.c_void_p]
        L.lbo_time.restype = C.c_long
        L.lbo_destroy.argtypes = [C.c_void_p]
        L.lbo_destroy.restype = None
        L.lbo_threads.argtypes = []
        L.lbo_threads.restype = C.c_int
        L.lbo_set_threads.argtypes = [C.c_int]
        L.lbo_set_threads.restype = None
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(cfg: dict) -> _Params:
    """Convert a parameter dict (paper notation) into the oracle's struct."""
    p = _Params()
    p.lattice = int(cfg.get("lattice", D3Q19))
    p.nx, p.ny, p.nz = (int(v) for v in cfg["shape"])
    p.alpha = _d2(*cfg.get("alpha", (1 / 3, 1 / 3)))
    p.rho0 = _d2(*cfg.get("rho0", (1.0, 1.0)))
    p.A = cfg.get("A", 0.05)
    p.beta = cfg.get("beta", 0.7)
    p.eps_g = cfg.get("eps_g", 1e-6)
    p.tau_b = cfg["tau_b"]
    p.rheology = _RHEO[cfg.get("rheology", "newtonian")]
    p.tau_y = cfg.get("tau_y", cfg["tau_b"])
    p.K = cfg.get("K", 0.0)
    p.n = cfg.get("n", 1.0)
    p.nu0 = cfg.get("nu0", 0.0)
    p.nu_inf = cfg.get("nu_inf", 0.0)
    p.lam = cfg.get("lambda", 0.0)
    p.m = cfg.get("m", 1.0)
    p.tau_min = cfg.get("tau_min", 0.51)
    p.tau_max = cfg.get("tau_max", 2.0)
    p.rho_eps = cfg.get("rho_eps", 1e-6)
    p.zeta_wall = _d2(*cfg.get("zeta_wall", (1.0, 1.0)))
    p.zeta_noz = _d2(*cfg.get("zeta_noz", (1.0, 1.0)))
    p.drag_gamma = cfg.get("drag_gamma", 0.0)
    p.drag_range = cfg.get("drag_range", 4.0)
    p.body_g = _d3(*cfg.get("body_g", (0.0, 0.0, 0.0)))
    p.face_zlo = _FACE[cfg.get("face_zlo", "periodic")]
    p.face_zhi = _FACE[cfg.get("face_zhi", "periodic")]
    p.u_zlo = _d3(*cfg.get("u_zlo", (0.0, 0.0, 0.0)))
    p.u_zhi = _d3(*cfg.get("u_zhi", (0.0, 0.0, 0.0)))
    p.rho_zlo = _d2(*cfg.get("rho_zlo", (0.0, 1.0)))
    p.rho_zhi = _d2(*cfg.get("rho_zhi", (0.0, 1.0)))
    noz = cfg.get("nozzle")
    p.has_nozzle = 1 if noz else 0
    if noz:
        p.noz_x0 = _d2(*noz["x0"])
        p.noz_v = _d2(*noz.get("v", (0.0, 0.0)))
        p.noz_r_in = noz["r_in"]
        p.noz_wall = noz.get("wall", 2.0)
        p.noz_tip_z = noz["tip_z"]
        p.u_ink = _d3(*noz.get("u_ink", (0.0, 0.0, 0.0)))
        p.lid_rho_y = noz.get("lid_rho_y", 1.0)
    p.collide = int(cfg.get("collide", 1))
    return p


# ---------------------------------------------------------------- lattice info

def lattice(lat: int = D3Q19):
    D, Q = C.c_int(), C.c_int()
    c = np.zeros(19 * 3, dtype=np.int32)
    w = np.zeros(19)
    cs2 = C.c_double()
    rc = lib().lbo_lattice(lat, C.byref(D), C.byref(Q), c.ctypes.data_as(C.POINTER(C.c_int)), _dp(w), C.byref(cs2))
    assert rc == 0
    q = Q.value
    return {"D": D.value, "Q": q, "c": c[: 3 * q].reshape(q, 3).copy(), "w": w[:q].copy(), "cs2": cs2.value}


def phi(lat: int, alpha: float) -> np.ndarray:
    out = np.zeros(19)
    assert lib().lbo_phi(lat, alpha, _dp(out)) == 0
    return out[: lattice(lat)["Q"]]


def B(lat: int) -> np.ndarray:
    out = np.zeros(19)
    assert lib().lbo_B(lat, _dp(out)) == 0
    return out[: lattice(lat)["Q"]]


def partial_pressure(lat: int, alpha: float, rho: float) -> float:
    return lib().lbo_partial_pressure(lat, alpha, rho)


def feq(lat: int, alpha: float, rho: float, u) -> np.ndarray:
    uu = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(19)
    assert lib().lbo_feq(lat, alpha, rho, _dp(uu), _dp(out)) == 0
    return out[: lattice(lat)["Q"]]


def regularize(lat: int, alpha: float, rho: float, u, f) -> np.ndarray:
    uu = np.ascontiguousarray(u, dtype=np.float64)
    ff = np.zeros(19)
    ff[: len(f)] = f
    out = np.zeros(19)
    assert lib().lbo_regularize(lat, alpha, rho, _dp(uu), _dp(ff), _dp(out)) == 0
    return out[: len(f)]


def perturbation(lat: int, A: float, gradN, Fcg) -> np.ndarray:
    g = np.ascontiguousarray(gradN, dtype=np.float64)
    F = np.ascontiguousarray(Fcg, dtype=np.float64)
    out = np.zeros(19)
    assert lib().lbo_perturbation(lat, A, _dp(g), _dp(F), _dp(out)) == 0
    return out[: lattice(lat)["Q"]]


def recolour(lat: int, alpha, beta: float, eps_g: float, rhoY: float, rhoB: float, gradN, fstar):
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    g = np.ascontiguousarray(gradN, dtype=np.float64)
    fs = np.zeros(19)
    fs[: len(fstar)] = fstar
    fY = np.zeros(19)
    fB = np.zeros(19)
    assert lib().lbo_recolour(lat, _dp(a), beta, eps_g, rhoY, rhoB, _dp(g), _dp(fs), _dp(fY), _dp(fB)) == 0
    q = len(fstar)
    return fY[:q], fB[:q]


def tau_ink(cfg: dict, S: float, rhoY: float):
    p = make_params(cfg)
    g, t = C.c_double(), C.c_double()
    assert lib().lbo_tau_ink(C.byref(p), S, rhoY, C.byref(g), C.byref(t)) == 0
    return g.value, t.value


def wall_density(r0: float, r1: float, r2: float, has1: bool, has2: bool) -> float:
    return lib().lbo_wall_density(r0, r1, r2, int(has1), int(has2))


def gradient(lat: int, chi: np.ndarray) -> np.ndarray:
    """Eq. (lattgrad) at the interior nodes of a (nz, ny, nx) field."""
    chi = np.ascontiguousarray(chi, dtype=np.float64)
    nz, ny, nx = chi.shape
    out = np.zeros(chi.shape + (3,))
    assert lib().lbo_gradient(lat, nx, ny, nz, _dp(chi), _dp(out)) == 0
    return out


def threads() -> int:
    """Threads the oracle's parallel loops use."""
    return int(lib().lbo_threads())


def set_threads(n: int) -> None:
    lib().lbo_set_threads(int(n))


# ------------------------------------------------------------------ simulation

class OracleSim:
    """One FP64 oracle simulation.  Fields are numpy arrays of shape
    (nz, ny, nx); velocities (nz, ny, nx, 3)."""

    def __init__(self, cfg: dict, rho_y: np.ndarray, rho_b: np.ndarray, u: np.ndarray | None = None):
        self.cfg = cfg
        self.shape = tuple(int(v) for v in cfg["shape"])  # (nx, ny, nz)
        nx, ny, nz = self.shape
        self._p = make_params(cfg)
        ry = np.ascontiguousarray(rho_y, dtype=np.float64).reshape(nz, ny, nx)
        rb = np.ascontiguousarray(rho_b, dtype=np.float64).reshape(nz, ny, nx)
        uu = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(nz, ny, nx, 3)
        h = C.c_void_p()
        rc = lib().lbo_create(C.byref(self._p), _dp(ry), _dp(rb), None if uu is None else _dp(uu), C.byref(h))
        if rc != 0:
            raise ValueError(f"lbo_create failed ({rc})")
        self._h = h
        self.Q = lattice(self._p.lattice)["Q"]

    def step(self, n: int = 1) -> None:
        assert lib().lbo_step(self._h, int(n)) == 0

    @property
    def t(self) -> int:
        return int(lib().lbo_time(self._h))

    def moments(self):
        nx, ny, nz = self.shape
        ry = np.zeros((nz, ny, nx))
        rb = np.zeros((nz, ny, nx))
        u = np.zeros((nz, ny, nx, 3))
        cons = Conserved()
        assert lib().lbo_moments(self._h, _dp(ry), _dp(rb), _dp(u), C.byref(cons)) == 0
        return ry, rb, u, cons.as_dict()

    def get_f(self, k: int) -> np.ndarray:
        nx, ny, nz = self.shape
        out = np.zeros((self.Q, nz, ny, nx))
        assert lib().lbo_get_f(self._h, k, _dp(out)) == 0
        return out

    def set_f(self, k: int, f: np.ndarray) -> None:
        a = np.ascontiguousarray(f, dtype=np.float64)
        assert lib().lbo_set_f(self._h, k, _dp(a)) == 0

    def solid(self) -> np.ndarray:
        nx, ny, nz = self.shape
        out = np.zeros((nz, ny, nx), dtype=np.uint8)
        assert lib().lbo_solid(self._h, out.ctypes.data_as(C.POINTER(C.c_uint8))) == 0
        return out.astype(bool)

    def velocities(self) -> np.ndarray:
        c = np.zeros(19 * 3, dtype=np.int32)
        q = lib().lbo_velocity_index(self._h, c.ctypes.data_as(C.POINTER(C.c_int)))
        return c[: 3 * q].reshape(q, 3)

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().lbo_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
