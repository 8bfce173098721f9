"""Python binding of ``liblbprint.so`` (C ABI in ``include/lbprint.h``).

Argument marshalling only: every step of the method runs in the HIP kernels.
PyTorch provides the device workspace (a uint8 tensor) and the stream.  There
is no CPU fallback: a missing library or a missing GPU raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbprint.so")

LB_OK, LB_EINVAL, LB_ENOMEM, LB_EDEVICE, LB_EUNSTABLE, LB_ESTATE = 0, -1, -2, -3, -4, -5
STORAGE = {"f64": 0, "f32": 1, "bf16dev": 2, "f16dev": 3}
RHEOLOGY = {"newtonian": 0, "power_law": 1, "cross": 2}
FACE = {"periodic": 0, "wall": 1, "pressure": 2}

EXPORTS = ("lb_footprint", "lb_create", "lb_step", "lb_step_batch", "lb_moments", "lb_moments_noalloc", "lb_observe",
           "lb_time",
           "lb_timing", "lb_timing_read", "lb_destroy", "lb_strerror", "lb_last_error", "lb_batch_footprint",
           "lb_batch_create", "lb_batch_step", "lb_batch_destroy", "lb_batch_last_error")

_d2 = C.c_double * 2
_d3 = C.c_double * 3


class Params(C.Structure):
    """Mirror of ``lb_params``."""
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("storage", C.c_int),
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
        ("check_interval", C.c_int),
        ("lattice", C.c_int),
    ]


class Conserved(C.Structure):
    """Mirror of ``lb_conserved``."""
    _fields_ = [
        ("mass", _d2), ("mom", _d3),
        ("mass_wall", _d2), ("mass_open", _d2),
        ("mass_created", _d2), ("mass_deleted", _d2),
    ]

    def as_dict(self) -> dict:
        return {name: np.array(list(getattr(self, name))) for name, _ in self._fields_}


class Window(C.Structure):
    """Mirror of ``lb_window``."""
    _fields_ = [("x_lo", C.c_int), ("x_len", C.c_int), ("z_hi", C.c_int), ("y", C.c_int)]


class Observables(C.Structure):
    """Mirror of ``lb_observables``."""
    _fields_ = [("ink_area", C.c_double), ("height", C.c_double), ("width", C.c_double),
                ("coverage", C.c_double), ("dp_max", C.c_double), ("p0", C.c_double),
                ("substrate_ink", C.c_double)]

    def as_dict(self) -> dict:
        return {name: float(getattr(self, name)) for name, _ in self._fields_}


class LBError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None


def lib():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run paper_2102_02655_amd/build.py)")
        # Load PyTorch's HIP runtime first: the library then binds to that same
        # runtime (same soname), so torch's device memory and streams are
        # valid in its calls.  Loading the library first would bring in a
        # second runtime instance.
        import torch  # noqa: F401

        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.lb_footprint.argtypes = [C.POINTER(Params), C.POINTER(C.c_size_t)]
        L.lb_create.argtypes = [C.POINTER(Params), vp, vp, vp, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.lb_step.argtypes = [vp, C.c_int]
        L.lb_step_batch.argtypes = [C.POINTER(vp), C.POINTER(C.c_int), C.c_int]
        L.lb_moments.argtypes = [vp, vp, vp, vp, C.c_int, C.c_int, C.POINTER(Conserved)]
        L.lb_moments_noalloc.argtypes = [vp, vp, vp, vp, C.c_int, C.c_int, C.POINTER(Conserved)]
        L.lb_observe.argtypes = [vp, C.POINTER(Window), C.POINTER(Observables)]
        L.lb_time.argtypes = [vp]
        L.lb_time.restype = C.c_long
        L.lb_timing.argtypes = [vp, C.c_int]
        L.lb_timing_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_long)]
        L.lb_destroy.argtypes = [vp]
        L.lb_strerror.argtypes = [C.c_int]
        L.lb_strerror.restype = C.c_char_p
        L.lb_last_error.argtypes = [vp]
        L.lb_last_error.restype = C.c_char_p
        L.lb_batch_footprint.argtypes = [C.POINTER(C.c_size_t)]
        L.lb_batch_create.argtypes = [C.c_int, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.lb_batch_step.argtypes = [vp, C.POINTER(vp), C.POINTER(C.c_int), C.c_int]
        L.lb_batch_destroy.argtypes = [vp]
        L.lb_batch_last_error.argtypes = [vp]
        L.lb_batch_last_error.restype = C.c_char_p
        for f in ("lb_footprint", "lb_create", "lb_step", "lb_step_batch", "lb_moments", "lb_moments_noalloc",
                  "lb_observe", "lb_timing", "lb_timing_read", "lb_destroy", "lb_batch_footprint", "lb_batch_create",
                  "lb_batch_step", "lb_batch_destroy"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def make_params(cfg: dict, check_interval: int = 0) -> Params:
    """Convert a parameter dict (paper notation) into ``lb_params``."""
    p = Params()
    lat = int(cfg.get("lattice", 19))
    if lat not in (9, 19):
        raise ValueError("lattice must be 9 (D2Q9) or 19 (D3Q19)")
    p.nx, p.ny, p.nz = (int(v) for v in cfg["shape"])
    p.storage = STORAGE[cfg.get("storage", "f32")]
    p.alpha = _d2(*cfg.get("alpha", (1 / 3, 1 / 3)))
    p.rho0 = _d2(*cfg.get("rho0", (1.0, 1.0)))
    p.A = cfg.get("A", 0.05)
    p.beta = cfg.get("beta", 0.7)
    p.eps_g = cfg.get("eps_g", 1e-6)
    p.tau_b = cfg["tau_b"]
    p.rheology = RHEOLOGY[cfg.get("rheology", "newtonian")]
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
    p.face_zlo = FACE[cfg.get("face_zlo", "periodic")]
    p.face_zhi = FACE[cfg.get("face_zhi", "periodic")]
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
    p.check_interval = int(check_interval)
    p.lattice = lat
    return p


def _raise(status: int, handle=None):
    msg = lib().lb_last_error(handle)
    raise LBError(status, (msg or b"").decode() or lib().lb_strerror(status).decode())


def footprint(cfg: dict) -> int:
    """Device bytes one simulation of this configuration needs."""
    p = make_params(cfg)
    n = C.c_size_t()
    rc = lib().lb_footprint(C.byref(p), C.byref(n))
    if rc != LB_OK:
        _raise(rc)
    return int(n.value)


def step_batch(sims, nsteps) -> None:
    """Advance every Sim in `sims` by the matching count in `nsteps` (an int
    applies to all) in one batched call (one graph launch for the even part)."""
    n = len(sims)
    if isinstance(nsteps, int):
        nsteps = [nsteps] * n
    hs = (C.c_void_p * n)(*[s._h.value for s in sims])
    ks = (C.c_int * n)(*[int(k) for k in nsteps])
    rc = lib().lb_step_batch(hs, ks, n)
    if rc != LB_OK:
        _raise(rc, sims[0]._h)


def _require_gpu():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("the lbprint GPU library needs a ROCm GPU; none is visible")
    return torch


class Sim:
    """One GPU simulation.  Fields are numpy arrays of shape (nz, ny, nx);
    velocities (nz, ny, nx, 3)."""

    def __init__(self, cfg: dict, rho_y: np.ndarray, rho_b: np.ndarray, u: np.ndarray | None = None,
                 device: str = "cuda:0", check_interval: int = 0, stream=None):
        torch = _require_gpu()
        self.cfg = cfg
        self.shape = tuple(int(v) for v in cfg["shape"])
        nx, ny, nz = self.shape
        self.device = torch.device(device)
        self._p = make_params(cfg, check_interval)
        self.nbytes = footprint(cfg)
        self.ws = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = self.ws.data_ptr()
        self._ws_ptr = (ptr + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ry = np.ascontiguousarray(rho_y, dtype=np.float64).reshape(nz, ny, nx)
        rb = np.ascontiguousarray(rho_b, dtype=np.float64).reshape(nz, ny, nx)
        uu = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(nz, ny, nx, 3)
        h = C.c_void_p()
        rc = lib().lb_create(C.byref(self._p), ry.ctypes.data, rb.ctypes.data, None if uu is None else uu.ctypes.data,
                             self._ws_ptr, self.nbytes, self.stream.cuda_stream, C.byref(h))
        if rc != LB_OK:
            _raise(rc)
        self._h = h

    def step(self, n: int = 1) -> None:
        rc = lib().lb_step(self._h, int(n))
        if rc != LB_OK:
            _raise(rc, self._h)

    @property
    def t(self) -> int:
        return int(lib().lb_time(self._h))

    def moments(self, dtype=np.float64, allow_unstable: bool = False):
        """Host copies of rho_Y, rho_B, u and the FP64 conserved sums."""
        nx, ny, nz = self.shape
        ry = np.zeros((nz, ny, nx), dtype=dtype)
        rb = np.zeros((nz, ny, nx), dtype=dtype)
        u = np.zeros((nz, ny, nx, 3), dtype=dtype)
        cons = Conserved()
        code = 0 if np.dtype(dtype) == np.float64 else 1
        rc = lib().lb_moments(self._h, ry.ctypes.data, rb.ctypes.data, u.ctypes.data, 0, code, C.byref(cons))
        if rc != LB_OK and not (allow_unstable and rc == LB_EUNSTABLE):
            _raise(rc, self._h)
        return ry, rb, u, cons.as_dict()

    def moments_device(self, ry, rb, u, dtype_code: int = 1):
        """Write the fields into caller-owned device tensors (no host copy of
        the fields); returns the conserved sums."""
        cons = Conserved()
        ptr = lambda t: None if t is None else t.data_ptr()  # noqa: E731
        rc = lib().lb_moments(self._h, ptr(ry), ptr(rb), ptr(u), 1, dtype_code, C.byref(cons))
        if rc != LB_OK:
            _raise(rc, self._h)
        return cons.as_dict()

    def observe(self, x_lo: int, x_len: int, z_hi: int, y: int = 0) -> dict:
        """Printing observables (lb_observe) of the section y: the thread in
        columns x_lo .. x_lo + x_len - 1 below z_hi, and the section's ink
        pressure and substrate contact."""
        w = Window(int(x_lo), int(x_len), int(z_hi), int(y))
        o = Observables()
        rc = lib().lb_observe(self._h, C.byref(w), C.byref(o))
        if rc != LB_OK:
            _raise(rc, self._h)
        return o.as_dict()

    def timing(self, enable: bool = True) -> None:
        """Start (or stop) HIP-event timing of the step kernels."""
        rc = lib().lb_timing(self._h, 1 if enable else 0)
        if rc != LB_OK:
            _raise(rc, self._h)

    def timing_read(self) -> dict:
        """Summed durations (ms) of the fused step kernel and of the boundary
        preparation kernels over the timed steps; clears the record."""
        a, b, n = C.c_double(), C.c_double(), C.c_long()
        rc = lib().lb_timing_read(self._h, C.byref(a), C.byref(b), C.byref(n))
        if rc != LB_OK:
            _raise(rc, self._h)
        return {"step_ms": a.value, "prep_ms": b.value, "steps": int(n.value)}

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().lb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A batch of simulations of one storage form stepped together: each
    call of step() advances every member (at most MAX_MEMBERS) by its own
    step count with one graph launch of the batched kernels over the device
    slot table (the workspace is a torch uint8 tensor; the stream the
    batch's own)."""

    MAX_MEMBERS = 64  # slots of the device table (lb_batch_step's limit)

    def __init__(self, storage: str = "f32", device: str = "cuda:0", stream=None):
        torch = _require_gpu()
        self.device = torch.device(device)
        self.storage = storage
        n = C.c_size_t()
        rc = lib().lb_batch_footprint(C.byref(n))
        if rc != LB_OK:
            _raise(rc)
        self.nbytes = int(n.value)
        self.ws = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.ws.data_ptr() + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        h = C.c_void_p()
        rc = lib().lb_batch_create(STORAGE[storage], ptr, self.nbytes, self.stream.cuda_stream, C.byref(h))
        if rc != LB_OK:
            _raise(rc)
        self._b = h

    def step(self, sims, nsteps) -> None:
        """Advance sims[i] by nsteps[i] steps (an int applies to all)."""
        n = len(sims)
        if isinstance(nsteps, int):
            nsteps = [nsteps] * n
        hs = (C.c_void_p * max(n, 1))(*[s._h.value for s in sims])
        ks = (C.c_int * max(n, 1))(*[int(k) for k in nsteps])
        rc = lib().lb_batch_step(self._b, hs, ks, n)
        if rc != LB_OK:
            msg = lib().lb_batch_last_error(self._b)
            raise LBError(rc, (msg or b"").decode() or lib().lb_strerror(rc).decode())

    def close(self) -> None:
        if getattr(self, "_b", None):
            lib().lb_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
