"""FP64 CPU oracle of the generalized single-phase LB model with a mass source (arXiv:1902.08933,
Sec. 2: eqs. 24, 25, 27, 27aa, 27a, 28 in the reductions of Remarks 1 and 3).

TEST INFRASTRUCTURE: ctypes wrapper over the ``sp_*`` functions of ``liblbpf_oracle.so``
(``oracle/sp_oracle.c``). It shares no code with the HIP library.
"""
import ctypes

import numpy as np

from . import _load as _load_base

NQ = 9
MODELS = {"nearly_incompressible": 0, "incompressible": 1}
FIELDS = {"rho": 0, "ux": 1, "uy": 2, "p": 3}
_D = ctypes.c_double
_PD = ctypes.POINTER(ctypes.c_double)


class SpParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("model", ctypes.c_int32),
                ("pscheme", ctypes.c_int32), ("full", ctypes.c_int32), ("bc", ctypes.c_int32),
                ("nu", _D), ("xi", _D), ("rho0", _D), ("drag", _D), ("scheme", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    lib = _load_base()
    lib.sp_create.restype = ctypes.c_void_p
    lib.sp_create.argtypes = [ctypes.POINTER(SpParams)]
    lib.sp_destroy.argtypes = [ctypes.c_void_p]
    lib.sp_init.argtypes = [ctypes.c_void_p] + [_PD] * 6
    lib.sp_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
    lib.sp_step_count.restype = ctypes.c_int64
    lib.sp_step_count.argtypes = [ctypes.c_void_p]
    lib.sp_read.argtypes = [ctypes.c_void_p, ctypes.c_int, _PD]
    lib.sp_read_force_distribution.argtypes = [ctypes.c_void_p, _PD]
    lib.sp_sum_rho_tilde.restype = _D
    lib.sp_sum_rho_tilde.argtypes = [ctypes.c_void_p]
    lib.sp_get_state.argtypes = [ctypes.c_void_p, _PD]
    lib.sp_force_distribution.argtypes = [_D] * 6 + [_PD]
    lib.sp_bracket.argtypes = [_D] * 8 + [_PD] * 3
    lib.sp_equilibrium_ni.argtypes = [_D] * 3 + [_PD]
    lib.sp_equilibrium_inc.argtypes = [_D] * 4 + [_PD]
    lib.sp_pressure_inc.restype = _D
    lib.sp_pressure_inc.argtypes = [_PD] + [_D] * 5 + [ctypes.c_int]
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_PD)


def _f64(a, n=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def make_params(cfg):
    """SpParams from a workload dict (keys as in paper_1902_08933_amd.workloads.single_phase_*)."""
    p = SpParams()
    p.nx, p.ny = int(cfg["nx"]), int(cfg["ny"])
    p.model = MODELS[cfg["model"]]
    p.pscheme = {"eq28": 0, "eq29": 1}[cfg.get("pscheme", "eq28")]
    p.full = int(bool(cfg.get("full", True)))
    p.bc = {"periodic": 0, "walls_y": 1}[cfg.get("bc", "periodic")]
    p.nu = float(cfg["nu"])
    p.xi = float(cfg.get("xi", 0.0))
    p.rho0 = float(cfg.get("rho0", 1.0))
    p.drag = float(cfg.get("drag", 0.0))
    p.scheme = {"eq24": 0, "remark4": 1}[cfg.get("scheme", "eq24")]
    return p


class SpOracle:
    """One FP64 single-phase simulation: init, step N, read rho/u/p."""

    def __init__(self, cfg):
        self.lib = _load()
        self.params = make_params(cfg)
        self.nx, self.ny = self.params.nx, self.params.ny
        self.n = self.nx * self.ny
        h = self.lib.sp_create(ctypes.byref(self.params))
        if not h:
            raise ValueError("invalid single-phase oracle parameters")
        self._h = ctypes.c_void_p(h)

    def __del__(self):
        if getattr(self, "_h", None) is not None and self.lib is not None:
            self.lib.sp_destroy(self._h)
            self._h = None

    def init(self, a0=None, ux=None, uy=None, S=None, Fx=None, Fy=None):
        """a0: initial density (model 0) or pressure (model 1); None: 1 or 0"""
        arrs = [_f64(a, self.n) for a in (a0, ux, uy, S, Fx, Fy)]
        self._keep = arrs
        self.lib.sp_init(self._h, *[_ptr(a) for a in arrs])
        return self

    def step(self, n=1):
        self.lib.sp_step(self._h, int(n))
        return self

    @property
    def step_count(self):
        return int(self.lib.sp_step_count(self._h))

    def read(self, field):
        out = np.empty(self.n)
        if self.lib.sp_read(self._h, FIELDS[field], _ptr(out)) != 0:
            raise ValueError(field)
        return out.reshape(self.ny, self.nx)

    def force_distribution(self):
        out = np.empty(NQ * self.n)
        self.lib.sp_read_force_distribution(self._h, _ptr(out))
        return out.reshape(NQ, self.ny, self.nx)

    def sum_rho_tilde(self):
        return float(self.lib.sp_sum_rho_tilde(self._h))

    def populations(self):
        out = np.empty(NQ * self.n)
        self.lib.sp_get_state(self._h, _ptr(out))
        return out.reshape(NQ, self.ny, self.nx)


def force_distribution(S, Fx, Fy, axx, axy, ayy):
    out = np.empty(NQ)
    _load().sp_force_distribution(S, Fx, Fy, axx, axy, ayy, _ptr(out))
    return out


def bracket(dtp, ux, uy, Ftx, Fty, St, Q, divu):
    a = [ctypes.c_double() for _ in range(3)]
    _load().sp_bracket(dtp, ux, uy, Ftx, Fty, St, Q, divu, *[ctypes.byref(x) for x in a])
    return tuple(x.value for x in a)


def equilibrium_ni(rho, ux, uy):
    out = np.empty(NQ)
    _load().sp_equilibrium_ni(rho, ux, uy, _ptr(out))
    return out


def equilibrium_inc(rho0, p, ux, uy):
    out = np.empty(NQ)
    _load().sp_equilibrium_inc(rho0, p, ux, uy, _ptr(out))
    return out


def pressure_inc(g, S, ux, uy, tau, G0, scheme=0):
    g = _f64(g, NQ)
    return float(_load().sp_pressure_inc(_ptr(g), S, ux, uy, tau, G0, int(scheme)))
