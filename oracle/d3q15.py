"""FP64 CPU oracle of the phase-field LB model on the D3Q15 lattice (arXiv:1902.08933).

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg of the benchmark
use this module. It wraps the ``o3_*`` functions of ``liblbpf_oracle.so`` (``d3q15_oracle.c``,
plain C in double precision) and shares no code with the HIP library. Arrays are [nz][ny][nx].
What pins each function is in ``tests/test_d3q15_oracle.py``.
"""
import ctypes

import numpy as np

from . import _load as _load2d, VARIANTS, PSCHEMES, FSURF, VISC

Q = 15
FIELDS = {"phi": 0, "rho": 1, "ux": 2, "uy": 3, "uz": 4, "p": 5, "mu": 6, "lap_phi": 7,
          "grad_phi_x": 8, "grad_phi_y": 9, "grad_phi_z": 10, "S": 11, "Fx": 12, "Fy": 13,
          "Fz": 14, "tau_g": 15}
BCS = {"periodic": 0, "walls_z": 1}


class O3Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("pscheme", ctypes.c_int32), ("fsurf", ctypes.c_int32),
                ("visc", ctypes.c_int32), ("bc", ctypes.c_int32), ("clamp_props", ctypes.c_int32),
                ("pad", ctypes.c_int32)] + \
               [(k, ctypes.c_double) for k in ("rho_A", "rho_B", "nu_A", "nu_B", "sigma", "W",
                                               "M_phi", "tau_h", "force_x", "force_y", "force_z",
                                               "gravity")]


_lib = None
_D = ctypes.c_double
_PD = ctypes.POINTER(ctypes.c_double)
_PP = ctypes.POINTER(O3Params)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    lib = _load2d()
    lib.o3_create.restype = ctypes.c_void_p
    lib.o3_create.argtypes = [_PP]
    lib.o3_destroy.argtypes = [ctypes.c_void_p]
    lib.o3_init.argtypes = [ctypes.c_void_p, _PD, _PD, _PD, _PD, _PD]
    lib.o3_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
    lib.o3_step_count.restype = ctypes.c_int64
    lib.o3_step_count.argtypes = [ctypes.c_void_p]
    lib.o3_read.argtypes = [ctypes.c_void_p, ctypes.c_int, _PD]
    lib.o3_get_state.argtypes = [ctypes.c_void_p, _PD, _PD, _PD, _PD]
    lib.o3_set_state.argtypes = [ctypes.c_void_p, _PD, _PD, _PD, _PD]
    lib.o3_sum_phi.restype = _D
    lib.o3_sum_phi.argtypes = [ctypes.c_void_p]
    lib.o3_laplace_pressure.argtypes = [ctypes.c_void_p, _PD]
    lib.o3_gradient.argtypes = [_PP, _PD, _PD, _PD, _PD]
    lib.o3_laplacian.argtypes = [_PP, _PD, _PD]
    lib.o3_equilibrium_g.argtypes = [_D, _D, _PD, _PD]
    lib.o3_equilibrium_h.argtypes = [_D, _D, _D, _PD, _PD]
    lib.o3_force_distribution.argtypes = [_D, _PD, _PD, _PD, _D, _D, _PD]
    lib.o3_G0_simplified.restype = _D
    lib.o3_G0_simplified.argtypes = [_D, _PD, _PD, _PD, _D]
    lib.o3_source_R.argtypes = [_D, _PD, _PD, _PD]
    lib.o3_pressure.restype = _D
    lib.o3_pressure.argtypes = [_PD, _D, _D, _PD, _D, _D, ctypes.c_int]
    lib.o3_lattice.argtypes = [ctypes.POINTER(ctypes.c_int32), _PD]
    lib.o3_density.restype = _D
    lib.o3_density.argtypes = [_PP, _D]
    lib.o3_viscosity.restype = _D
    lib.o3_viscosity.argtypes = [_PP, _D]
    _lib = lib
    return lib


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def _ptr(a):
    return a.ctypes.data_as(_PD)


def _vec(v):
    return _f64(np.asarray(v, dtype=np.float64).reshape(3))


def make_params(cfg):
    p = O3Params()
    p.nx, p.ny, p.nz = int(cfg["nx"]), int(cfg["ny"]), int(cfg["nz"])
    p.variant = VARIANTS[cfg.get("variant", "qim")]
    p.pscheme = PSCHEMES[cfg.get("pscheme", "eq28")]
    p.fsurf = FSURF[cfg.get("fsurf", "mu_grad_phi")]
    p.visc = VISC[cfg.get("visc", "inverse_linear")]
    p.bc = BCS[cfg.get("bc", "periodic")]
    p.clamp_props = int(bool(cfg.get("clamp_props", False)))
    for k in ("rho_A", "rho_B", "nu_A", "nu_B", "sigma", "W", "M_phi", "tau_h"):
        setattr(p, k, float(cfg[k]))
    for k in ("force_x", "force_y", "force_z", "gravity"):
        setattr(p, k, float(cfg.get(k, 0.0)))
    return p


class Oracle3D:
    """One FP64 D3Q15 simulation on the CPU."""

    def __init__(self, cfg):
        self.lib = _load()
        self.params = make_params(cfg)
        self.shape = (self.params.nz, self.params.ny, self.params.nx)
        self.n = int(np.prod(self.shape))
        h = self.lib.o3_create(ctypes.byref(self.params))
        if not h:
            raise ValueError("invalid oracle parameters")
        self._h = ctypes.c_void_p(h)

    def __del__(self):
        if getattr(self, "_h", None) is not None and self.lib is not None:
            self.lib.o3_destroy(self._h)
            self._h = None

    def init(self, phi, ux=None, uy=None, uz=None, p=None):
        arrs = [_f64(phi, self.n)] + [None if a is None else _f64(a, self.n) for a in (ux, uy, uz, p)]
        self._keep = arrs
        self.lib.o3_init(self._h, *[None if a is None else _ptr(a) for a in arrs])
        return self

    def step(self, n=1):
        self.lib.o3_step(self._h, int(n))
        return self

    @property
    def step_count(self):
        return int(self.lib.o3_step_count(self._h))

    def read(self, field):
        out = np.empty(self.n)
        if self.lib.o3_read(self._h, FIELDS[field], _ptr(out)) != 0:
            raise ValueError(field)
        return out.reshape(self.shape)

    def get_state(self):
        g = np.empty(Q * self.n); h = np.empty(Q * self.n)
        pu = np.empty(3 * self.n); pp = np.empty(self.n)
        self.lib.o3_get_state(self._h, _ptr(g), _ptr(h), _ptr(pu), _ptr(pp))
        return (g.reshape((Q,) + self.shape), h.reshape((Q,) + self.shape),
                pu.reshape((3,) + self.shape), pp.reshape(self.shape))

    def set_state(self, g, h, phiu_prev, p_prev):
        a = [_f64(g, Q * self.n), _f64(h, Q * self.n), _f64(phiu_prev, 3 * self.n),
             _f64(p_prev, self.n)]
        self.lib.o3_set_state(self._h, *[_ptr(x) for x in a])

    def sum_phi(self):
        return float(self.lib.o3_sum_phi(self._h))

    def laplace_pressure(self):
        out = np.empty(self.n)
        self.lib.o3_laplace_pressure(self._h, _ptr(out))
        return out.reshape(self.shape)


# ---- per-node and per-field functions, exposed for the pinning tests -----------------------

def lattice():
    c = np.empty(3 * Q, dtype=np.int32); w = np.empty(Q)
    _load().o3_lattice(c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _ptr(w))
    return c.reshape(Q, 3), w


def _grid_params(z, bc):
    nz, ny, nx = z.shape
    return make_params(dict(nx=nx, ny=ny, nz=nz, bc=bc, rho_A=1, rho_B=1, nu_A=0.1, nu_B=0.1,
                            sigma=0, W=4, M_phi=0.1, tau_h=1))


def gradient(z, bc="periodic"):
    z = _f64(z)
    p = _grid_params(z, bc)
    g = [np.empty_like(z) for _ in range(3)]
    _load().o3_gradient(ctypes.byref(p), _ptr(z), *[_ptr(a) for a in g])
    return g


def laplacian(z, bc="periodic"):
    z = _f64(z)
    p = _grid_params(z, bc)
    out = np.empty_like(z)
    _load().o3_laplacian(ctypes.byref(p), _ptr(z), _ptr(out))
    return out


def equilibrium_g(p, rho, u):
    out = np.empty(Q)
    _load().o3_equilibrium_g(p, rho, _ptr(_vec(u)), _ptr(out))
    return out


def equilibrium_h(phi, mu, eta, u):
    out = np.empty(Q)
    _load().o3_equilibrium_h(phi, mu, eta, _ptr(_vec(u)), _ptr(out))
    return out


def force_distribution(rho, u, F, Ft, S, S1):
    out = np.empty(Q)
    u, F, Ft = _vec(u), _vec(F), _vec(Ft)
    _load().o3_force_distribution(rho, _ptr(u), _ptr(F), _ptr(Ft), S, S1, _ptr(out))
    return out


def G0_simplified(rho, u, F, gp, S1):
    u, F, gp = _vec(u), _vec(F), _vec(gp)
    return _load().o3_G0_simplified(rho, _ptr(u), _ptr(F), _ptr(gp), S1)


def source_R(tau_h, phiu, phiu_prev):
    out = np.empty(Q)
    a, b = _vec(phiu), _vec(phiu_prev)
    _load().o3_source_R(tau_h, _ptr(a), _ptr(b), _ptr(out))
    return out


def pressure(g, S, rho, u, tau_g, G0, with_G0=True):
    g = _f64(g, Q)
    return _load().o3_pressure(_ptr(g), S, rho, _ptr(_vec(u)), tau_g, G0, int(bool(with_G0)))
