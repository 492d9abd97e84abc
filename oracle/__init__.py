"""FP64 CPU oracle of the phase-field lattice Boltzmann model (arXiv:1902.08933).

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg of the benchmark
use this package. It is a ctypes wrapper over ``liblbpf_oracle.so`` (plain C, double precision,
built from ``lbpf_oracle.c`` by ``oracle/build.py``) and shares no code with the HIP library.

Parity status of each oracle function (what pins it) is listed in the tests under
``tests/test_oracle_*.py``; every function listed here is pinned.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbpf_oracle.so")

NQ = 9
FIELDS = {"phi": 0, "rho": 1, "ux": 2, "uy": 3, "p": 4, "mu": 5, "lap_phi": 6,
          "grad_phi_x": 7, "grad_phi_y": 8, "S": 9, "Fx": 10, "Fy": 11, "tau_g": 12}

VARIANTS = {"qim": 0, "im": 1}
PSCHEMES = {"eq28": 0, "eq28_paper_g0": 1, "eq29": 2}
FSURF = {"mu_grad_phi": 0, "neg_phi_grad_mu": 1}
VISC = {"inverse_linear": 0, "step": 1}
BCS = {"periodic": 0, "walls_y": 1}


class OrcParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("pscheme", ctypes.c_int32), ("fsurf", ctypes.c_int32), ("visc", ctypes.c_int32),
                ("bc", ctypes.c_int32), ("clamp_props", ctypes.c_int32),
                ("rho_A", ctypes.c_double), ("rho_B", ctypes.c_double),
                ("nu_A", ctypes.c_double), ("nu_B", ctypes.c_double),
                ("sigma", ctypes.c_double), ("W", ctypes.c_double), ("M_phi", ctypes.c_double),
                ("tau_h", ctypes.c_double), ("force_x", ctypes.c_double),
                ("force_y", ctypes.c_double), ("gravity", ctypes.c_double)]


_lib = None
_D = ctypes.c_double
_PD = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(LIB_PATH)
    lib.orc_create.restype = ctypes.c_void_p
    lib.orc_create.argtypes = [ctypes.POINTER(OrcParams)]
    lib.orc_destroy.argtypes = [ctypes.c_void_p]
    lib.orc_init.argtypes = [ctypes.c_void_p, _PD, _PD, _PD, _PD]
    lib.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
    lib.orc_step_count.restype = ctypes.c_int64
    lib.orc_step_count.argtypes = [ctypes.c_void_p]
    lib.orc_read.argtypes = [ctypes.c_void_p, ctypes.c_int, _PD]
    lib.orc_read_force_distribution.argtypes = [ctypes.c_void_p, _PD]
    lib.orc_get_state.argtypes = [ctypes.c_void_p, _PD, _PD, _PD, _PD]
    lib.orc_set_state.argtypes = [ctypes.c_void_p, _PD, _PD, _PD, _PD]
    lib.orc_sum_phi.restype = _D
    lib.orc_sum_phi.argtypes = [ctypes.c_void_p]
    lib.orc_laplace_pressure.argtypes = [ctypes.c_void_p, _PD]
    lib.orc_derived.argtypes = [ctypes.c_void_p, _PD]
    lib.orc_gradient.argtypes = [ctypes.POINTER(OrcParams), _PD, _PD, _PD]
    lib.orc_laplacian.argtypes = [ctypes.POINTER(OrcParams), _PD, _PD]
    lib.orc_equilibrium_g.argtypes = [_D, _D, _D, _D, _PD]
    lib.orc_equilibrium_h.argtypes = [_D, _D, _D, _D, _D, _PD]
    lib.orc_force_distribution.argtypes = [_D] * 9 + [_PD]
    lib.orc_G0_simplified.restype = _D
    lib.orc_G0_simplified.argtypes = [_D] * 8
    lib.orc_source_R.argtypes = [_D] * 5 + [_PD]
    lib.orc_pressure.restype = _D
    lib.orc_pressure.argtypes = [_PD, _D, _D, _D, _D, _D, _D, ctypes.c_int]
    lib.orc_free_energy_coeffs.argtypes = [_D, _D, _PD, _PD]
    lib.orc_eta.restype = _D
    lib.orc_eta.argtypes = [_D, _D]
    lib.orc_gamma.restype = _D
    lib.orc_gamma.argtypes = [_D, _D]
    lib.orc_density.restype = _D
    lib.orc_density.argtypes = [ctypes.POINTER(OrcParams), _D]
    lib.orc_viscosity.restype = _D
    lib.orc_viscosity.argtypes = [ctypes.POINTER(OrcParams), _D]
    lib.orc_chemical_potential.restype = _D
    lib.orc_chemical_potential.argtypes = [_D, _D, _D, _D]
    lib.orc_params_valid.restype = ctypes.c_int
    lib.orc_params_valid.argtypes = [ctypes.POINTER(OrcParams)]
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(_PD)


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def make_params(cfg):
    """OrcParams from a workload dict (keys as in paper_1902_08933_amd.workloads)."""
    p = OrcParams()
    p.nx, p.ny = int(cfg["nx"]), int(cfg["ny"])
    p.variant = VARIANTS[cfg.get("variant", "qim")]
    p.pscheme = PSCHEMES[cfg.get("pscheme", "eq28")]
    p.fsurf = FSURF[cfg.get("fsurf", "mu_grad_phi")]
    p.visc = VISC[cfg.get("visc", "inverse_linear")]
    p.bc = BCS[cfg.get("bc", "periodic")]
    p.clamp_props = int(bool(cfg.get("clamp_props", False)))
    for k in ("rho_A", "rho_B", "nu_A", "nu_B", "sigma", "W", "M_phi", "tau_h"):
        setattr(p, k, float(cfg[k]))
    p.force_x = float(cfg.get("force_x", 0.0))
    p.force_y = float(cfg.get("force_y", 0.0))
    p.gravity = float(cfg.get("gravity", 0.0))
    return p


class Oracle:
    """One FP64 simulation on the CPU: init fields, step N, read phi/rho/u/p/mu."""

    def __init__(self, cfg):
        self.lib = _load()
        self.params = make_params(cfg)
        self.nx, self.ny = self.params.nx, self.params.ny
        self.n = self.nx * self.ny
        h = self.lib.orc_create(ctypes.byref(self.params))
        if not h:
            raise ValueError("invalid oracle parameters")
        self._h = ctypes.c_void_p(h)

    def __del__(self):
        if getattr(self, "_h", None) is not None and self.lib is not None:
            self.lib.orc_destroy(self._h)
            self._h = None

    def init(self, phi, ux=None, uy=None, p=None):
        arrs = [_f64(phi, self.n)] + [None if a is None else _f64(a, self.n) for a in (ux, uy, p)]
        ptrs = [None if a is None else _ptr(a) for a in arrs]
        self._keep = arrs
        self.lib.orc_init(self._h, *ptrs)
        return self

    def step(self, n=1):
        self.lib.orc_step(self._h, int(n))
        return self

    @property
    def step_count(self):
        return int(self.lib.orc_step_count(self._h))

    def read(self, field):
        out = np.empty(self.n, dtype=np.float64)
        if self.lib.orc_read(self._h, FIELDS[field], _ptr(out)) != 0:
            raise ValueError(field)
        return out.reshape(self.ny, self.nx)

    def force_distribution(self):
        out = np.empty(NQ * self.n, dtype=np.float64)
        self.lib.orc_read_force_distribution(self._h, _ptr(out))
        return out.reshape(NQ, self.ny, self.nx)

    def get_state(self):
        g = np.empty(NQ * self.n); h = np.empty(NQ * self.n)
        pu = np.empty(2 * self.n); pp = np.empty(self.n)
        self.lib.orc_get_state(self._h, _ptr(g), _ptr(h), _ptr(pu), _ptr(pp))
        s = (self.ny, self.nx)
        return (g.reshape((NQ,) + s), h.reshape((NQ,) + s), pu.reshape((2,) + s), pp.reshape(s))

    def set_state(self, g, h, phiu_prev, p_prev):
        a = [_f64(g, NQ * self.n), _f64(h, NQ * self.n), _f64(phiu_prev, 2 * self.n),
             _f64(p_prev, self.n)]
        self.lib.orc_set_state(self._h, *[_ptr(x) for x in a])

    def sum_phi(self):
        return float(self.lib.orc_sum_phi(self._h))

    def laplace_pressure(self):
        out = np.empty(self.n, dtype=np.float64)
        self.lib.orc_laplace_pressure(self._h, _ptr(out))
        return out.reshape(self.ny, self.nx)

    def derived(self):
        out = np.empty(4)
        self.lib.orc_derived(self._h, _ptr(out))
        return dict(beta=out[0], kappa=out[1], eta=out[2], gamma=out[3])


# ---- per-cell and per-field functions, exposed for the pinning tests -----------------------

def gradient(z, bc="periodic"):
    z = _f64(z)
    ny, nx = z.shape
    p = make_params(dict(nx=nx, ny=ny, bc=bc, rho_A=1, rho_B=1, nu_A=0.1, nu_B=0.1, sigma=0,
                         W=4, M_phi=0.1, tau_h=1))
    gx = np.empty_like(z); gy = np.empty_like(z)
    _load().orc_gradient(ctypes.byref(p), _ptr(z), _ptr(gx), _ptr(gy))
    return gx, gy


def laplacian(z, bc="periodic"):
    z = _f64(z)
    ny, nx = z.shape
    p = make_params(dict(nx=nx, ny=ny, bc=bc, rho_A=1, rho_B=1, nu_A=0.1, nu_B=0.1, sigma=0,
                         W=4, M_phi=0.1, tau_h=1))
    out = np.empty_like(z)
    _load().orc_laplacian(ctypes.byref(p), _ptr(z), _ptr(out))
    return out


def equilibrium_g(p, rho, ux, uy):
    out = np.empty(NQ)
    _load().orc_equilibrium_g(p, rho, ux, uy, _ptr(out))
    return out


def equilibrium_h(phi, mu, eta, ux, uy):
    out = np.empty(NQ)
    _load().orc_equilibrium_h(phi, mu, eta, ux, uy, _ptr(out))
    return out


def force_distribution(rho, ux, uy, Fx, Fy, Ftx, Fty, S, S1):
    out = np.empty(NQ)
    _load().orc_force_distribution(rho, ux, uy, Fx, Fy, Ftx, Fty, S, S1, _ptr(out))
    return out


def G0_simplified(rho, ux, uy, Fx, Fy, gpx, gpy, S1):
    return _load().orc_G0_simplified(rho, ux, uy, Fx, Fy, gpx, gpy, S1)


def source_R(tau_h, phiux, phiuy, phiux_prev, phiuy_prev):
    out = np.empty(NQ)
    _load().orc_source_R(tau_h, phiux, phiuy, phiux_prev, phiuy_prev, _ptr(out))
    return out


def pressure(g, S, rho, ux, uy, tau_g, G0, with_G0=True):
    g = _f64(g, NQ)
    return _load().orc_pressure(_ptr(g), S, rho, ux, uy, tau_g, G0, int(bool(with_G0)))


def free_energy_coeffs(sigma, W):
    b = ctypes.c_double(); k = ctypes.c_double()
    _load().orc_free_energy_coeffs(sigma, W, ctypes.byref(b), ctypes.byref(k))
    return b.value, k.value


def eta(M_phi, tau_h):
    return _load().orc_eta(M_phi, tau_h)


def gamma(rho_A, rho_B):
    return _load().orc_gamma(rho_A, rho_B)


def chemical_potential(beta, kappa, phi, lap_phi):
    return _load().orc_chemical_potential(beta, kappa, phi, lap_phi)


def density(cfg, phi):
    p = make_params(dict(cfg, nx=cfg.get("nx", 3), ny=cfg.get("ny", 3)))
    return _load().orc_density(ctypes.byref(p), phi)


def viscosity(cfg, phi):
    p = make_params(dict(cfg, nx=cfg.get("nx", 3), ny=cfg.get("ny", 3)))
    return _load().orc_viscosity(ctypes.byref(p), phi)
