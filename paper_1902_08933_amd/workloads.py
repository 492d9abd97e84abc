"""Seeded synthetic workloads: physical parameters and initial order-parameter fields.

This module holds inputs only. It contains none of the method's arithmetic (no equilibria,
stencils, closures or derived coefficients); both the HIP library and the CPU oracle receive the
same arrays from here. Parameters are the raw physical ones of the paper's problem statement
(densities, viscosities, surface tension, interface width, mobility, tau_h, forces); each side
derives its own model coefficients from them.

Coordinates: nodes at integer (i, j), 0-based, x = i fastest, arrays shaped [ny, nx].
Order parameter convention of the paper: phi = 1 is phase A, phi = 0 is phase B (Sec. 3.1).
"""
import math

import numpy as np

# common defaults of every workload dict
BASE = dict(variant="qim", pscheme="eq28", fsurf="mu_grad_phi", visc="inverse_linear",
            bc="periodic", clamp_props=False, force_x=0.0, force_y=0.0, gravity=0.0)


def nu_from_tau(tau):
    """Kinematic viscosity of a BGK relaxation time (lattice units, c_s^2 = 1/3)."""
    return (tau - 0.5) / 3.0


def _cfg(**kw):
    c = dict(BASE)
    c.update(kw)
    return c


# ---- initial fields ------------------------------------------------------------------------

def droplet_phi(nx, ny, R, W, xc=None, yc=None, inside=1.0):
    """Circular interface profile of the static-droplet test (Sec. 4.2, eq. 36):
    phi = 1/2 + 1/2 tanh(2 (R - r) / W), centre at (nx/2, ny/2) unless given, periodic distance.
    inside=0 gives a bubble of phase B in phase A."""
    xc = nx / 2.0 if xc is None else xc
    yc = ny / 2.0 if yc is None else yc
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    dx = x - xc
    dy = y - yc
    r = np.sqrt(dx * dx + dy * dy)
    prof = 0.5 + 0.5 * np.tanh(2.0 * (R - r) / W)
    return prof if inside == 1.0 else 1.0 - prof


def periodic_droplet_phi(nx, ny, R, W, xc=None, yc=None):
    """Droplet profile with the minimum-image (periodic) distance to the centre."""
    xc = nx / 2.0 if xc is None else xc
    yc = ny / 2.0 if yc is None else yc
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    dx = np.abs(x - xc); dx = np.minimum(dx, nx - dx)
    dy = np.abs(y - yc); dy = np.minimum(dy, ny - dy)
    r = np.sqrt(dx * dx + dy * dy)
    return 0.5 + 0.5 * np.tanh(2.0 * (R - r) / W)


def spinodal_phi(nx, ny, mean, amplitude, seed):
    """Homogeneous mixture plus seeded uniform noise on [-amplitude, amplitude] (Sec. 4.1)."""
    rng = np.random.default_rng(seed)
    return mean + rng.uniform(-amplitude, amplitude, size=(ny, nx))


def layered_phi(nx, ny, W):
    """Layered channel (Sec. 4.3): walls half a cell below row 0 and above row ny-1, channel
    coordinate y = j + 1/2 - ny/2 in [-h, h] with h = ny/2; fluid A (phi = 1) on top."""
    y = np.arange(ny, dtype=np.float64)[:, None] + 0.5 - ny / 2.0
    return np.broadcast_to(0.5 + 0.5 * np.tanh(2.0 * y / W), (ny, nx)).copy()


def plane_phi(nx, ny, W, y0=None):
    """Flat interface along x at height y0 (equilibrium profile of eq. 9), A above."""
    y0 = ny / 2.0 if y0 is None else y0
    y = np.arange(ny, dtype=np.float64)[:, None] - y0
    return np.broadcast_to(0.5 + 0.5 * np.tanh(2.0 * y / W), (ny, nx)).copy()


# ---- workloads -----------------------------------------------------------------------------

def static_droplet(n=64, R=16.0, variant="qim", rho_ratio=10.0, sigma=0.01, tau=0.8,
                   tau_h=0.8, M_phi=0.02, W=4.0):
    """Static droplet: n x n periodic, droplet of phase A (heavy) centred, F_s = -phi grad mu
    (Sec. 4.2), rho_B = 1, tau_f = tau_h = 0.8, sigma = 0.01, M_phi = 0.02."""
    cfg = _cfg(name="static_droplet", nx=n, ny=n, variant=variant, fsurf="neg_phi_grad_mu",
               rho_A=rho_ratio, rho_B=1.0, nu_A=nu_from_tau(tau), nu_B=nu_from_tau(tau),
               sigma=sigma, W=W, M_phi=M_phi, tau_h=tau_h, R=R)
    phi = droplet_phi(n, n, R, W)
    return cfg, phi


def spinodal(n=1024, variant="qim", seed=0, rho_ratio=3.0, sigma=0.03, W=4.0, M_phi=0.1,
             tau_h=1.0, nu_B=1.0, nu_ratio=0.1, mean=0.5, amplitude=0.005):
    """Spinodal decomposition: n x n periodic, phi = 0.5 + U[-0.005, 0.005] (the +-1 order
    parameter 0 +- 0.01 mapped to [0, 1]), rho_A/rho_B = 3, nu_A/nu_B = 0.1, sigma = 0.03, W = 4,
    M_phi = 0.1, tau_h = 1 (Sec. 4.1 parameters with the density ratio of the workload).
    Sec. 4.1 gives only the viscosity ratio: nu_B = 1 (tau 3.5, and tau 0.8 for phase A) keeps the
    quasi-incompressible scheme finite over 20000 steps, where nu_B = 1/6 (tau_A = 0.55) goes
    non-finite after about 6000 steps, in FP64 as well."""
    cfg = _cfg(name="spinodal", nx=n, ny=n, variant=variant, rho_A=rho_ratio, rho_B=1.0,
               nu_A=nu_B * nu_ratio, nu_B=nu_B, sigma=sigma, W=W, M_phi=M_phi, tau_h=tau_h,
               seed=seed)
    phi = spinodal_phi(n, n, mean, amplitude, seed)
    return cfg, phi


def layered_poiseuille(nx=256, ny=128, mu_ratio=10.0, nu_B=0.1, G=1e-6, rho_ratio=1.0,
                       variant="qim", visc="inverse_linear", sigma=0.001, M_phi=0.1, W=4.0,
                       tau_h=1.0):
    """Layered Poiseuille flow (Sec. 4.3): periodic in x, halfway bounce-back walls in y,
    body force G along x, fluid A on top, mu_A/mu_B = mu_ratio."""
    rho_B = 1.0
    rho_A = rho_ratio * rho_B
    mu_B = rho_B * nu_B
    mu_A = mu_ratio * mu_B
    cfg = _cfg(name="layered_poiseuille", nx=nx, ny=ny, variant=variant, visc=visc,
               bc="walls_y", rho_A=rho_A, rho_B=rho_B, nu_A=mu_A / rho_A, nu_B=nu_B,
               sigma=sigma, W=W, M_phi=M_phi, tau_h=tau_h, force_x=G, mu_A=mu_A, mu_B=mu_B)
    phi = layered_phi(nx, ny, W)
    return cfg, phi


def rising_bubble(nx=512, ny=2048, R=64.0, rho_ratio=1000.0, sigma=0.01, eotvos=10.0,
                  reynolds=35.0, M_phi=0.02, tau_h=1.0, W=4.0, variant="qim"):
    """Rising bubble: phase-B bubble of radius R in phase A, periodic in x, walls in y,
    buoyancy F_y = -(rho - rho_A) g (Sec. 4.4), with g from Eo = (rho_A-rho_B) g (2R)^2/sigma
    and nu from Re = sqrt(g 2R) 2R / nu."""
    rho_A = 1.0
    rho_B = rho_A / rho_ratio
    D = 2.0 * R
    g = eotvos * sigma / ((rho_A - rho_B) * D * D)
    nu = math.sqrt(g * D) * D / reynolds
    cfg = _cfg(name="rising_bubble", nx=nx, ny=ny, variant=variant, bc="walls_y",
               clamp_props=True, rho_A=rho_A, rho_B=rho_B, nu_A=nu, nu_B=nu, sigma=sigma, W=W,
               M_phi=M_phi, tau_h=tau_h, gravity=g)
    phi = droplet_phi(nx, ny, R, W, xc=nx / 2.0, yc=4.0 * R, inside=0.0)
    return cfg, phi


def batch_instances(count=256, seed=0, side_min=64, side_max=512):
    """Independent instances for the batched step: square grids of side U{64..512}, alternating
    static droplet and layered Poiseuille; droplet radius U[0.15, 0.35] * side; density ratio
    log-uniform in [1, 1000]; viscosity ratio U[1, 100] with nu_B = 0.1; sigma U[1e-3, 1e-2];
    W = 4, M_phi = 0.02, tau_h = 0.8; Poiseuille force 1e-6 (64/side)^2."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        s = int(rng.integers(side_min, side_max + 1))
        rho_ratio = float(math.exp(rng.uniform(0.0, math.log(1000.0))))
        visc_ratio = float(rng.uniform(1.0, 100.0))
        sigma = float(rng.uniform(1e-3, 1e-2))
        frac = float(rng.uniform(0.15, 0.35))
        nu_B = 0.1
        if k % 2 == 0:
            cfg = _cfg(name="batch_droplet", nx=s, ny=s, fsurf="neg_phi_grad_mu",
                       rho_A=rho_ratio, rho_B=1.0, nu_A=nu_B * visc_ratio / rho_ratio,
                       nu_B=nu_B, sigma=sigma, W=4.0, M_phi=0.02, tau_h=0.8,
                       clamp_props=rho_ratio >= 100.0, R=frac * s)
            phi = droplet_phi(s, s, frac * s, 4.0)
        else:
            cfg = _cfg(name="batch_poiseuille", nx=s, ny=s, bc="walls_y", rho_A=rho_ratio,
                       rho_B=1.0, nu_A=nu_B * visc_ratio / rho_ratio, nu_B=nu_B, sigma=sigma,
                       W=4.0, M_phi=0.02, tau_h=0.8, force_x=1e-6 * (64.0 / s) ** 2,
                       clamp_props=rho_ratio >= 100.0)
            phi = layered_phi(s, s, 4.0)
        out.append((cfg, phi))
    return out


def single_phase_source(nx=1024, ny=1024, model="incompressible", S0=1e-4, F0=0.0, nu=1.0 / 6.0,
                        xi=0.0, full=True, bc="periodic", pscheme="eq28", seed=None, drag=0.0,
                        scheme="eq24"):
    """Single-phase flow driven by a mass source (Sec. 2): S = S0 sin(2 pi x/nx) cos(2 pi y/ny),
    a uniform force F0 in x (minus drag * rho u if drag > 0), fluid at rest; scheme "eq24" or
    "remark4" (Remark 4's explicit D_i G_i scheme, nearly incompressible model). With `seed`, the initial density (or pressure),
    velocity, source and force also carry small seeded smooth perturbations (parity cases).
    Returns (cfg, fields) with fields a dict of [ny, nx] float64 arrays (a0, ux, uy, S, Fx, Fy)."""
    cfg = dict(nx=nx, ny=ny, model=model, nu=nu, xi=xi, full=full, bc=bc, pscheme=pscheme, rho0=1.0,
               drag=drag, scheme=scheme)
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    S = S0 * np.sin(2 * np.pi * x / nx) * np.cos(2 * np.pi * y / ny)
    Fx = np.full((ny, nx), float(F0))
    Fy = np.zeros((ny, nx))
    a0 = np.ones((ny, nx)) if model == "nearly_incompressible" else np.zeros((ny, nx))
    ux = np.zeros((ny, nx))
    uy = np.zeros((ny, nx))
    if seed is not None:
        rng = np.random.default_rng(seed)

        def smooth(amp):
            # a few random Fourier modes of the grid
            f = np.zeros((ny, nx))
            for _ in range(4):
                kx, ky = rng.integers(1, 4, size=2)
                ph = rng.uniform(0, 2 * np.pi, size=2)
                f += np.sin(2 * np.pi * kx * x / nx + ph[0]) * np.cos(2 * np.pi * ky * y / ny + ph[1])
            return amp * f / 4

        a0 = a0 + smooth(1e-3)
        ux, uy = smooth(1e-3), smooth(1e-3)
        S = S + smooth(S0) + 0.2 * S0
        Fx, Fy = Fx + smooth(1e-5), smooth(1e-5)
    return cfg, dict(a0=a0, ux=ux, uy=uy, S=S, Fx=Fx, Fy=Fy)


# ---- three-dimensional workloads (D3Q15 solver): arrays shaped [nz, ny, nx] ----------------

BASE3D = dict(BASE, bc="periodic", force_z=0.0)


def spinodal3d(n=256, variant="qim", seed=0, rho_ratio=3.0, sigma=0.03, W=4.0, M_phi=0.01,
               tau_h=1.0, nu_B=1.0 / 6.0, nu_ratio=0.1, mean=0.5, amplitude=0.005, nz=None,
               ny=None):
    """Spinodal decomposition in a periodic n x n x n box (nz, ny override two sides): the
    two-dimensional spinodal workload's parameters, phi = mean + U[-amplitude, amplitude],
    except the mobility M_phi = 0.01 (the two-dimensional 0.1 makes the quasi-incompressible
    three-dimensional scheme unstable: velocities grow within tens of steps, in FP64 as well)."""
    nz = n if nz is None else nz
    ny = n if ny is None else ny
    cfg = dict(BASE3D, name="spinodal3d", nx=n, ny=ny, nz=nz, variant=variant, rho_A=rho_ratio,
               rho_B=1.0, nu_A=nu_B * nu_ratio, nu_B=nu_B, sigma=sigma, W=W, M_phi=M_phi,
               tau_h=tau_h, seed=seed)
    rng = np.random.default_rng(seed)
    phi = mean + rng.uniform(-amplitude, amplitude, size=(nz, ny, n))
    return cfg, phi


def sphere_phi(nx, ny, nz, R, W, centre=None, cylinder=False):
    """phi = 1/2 + 1/2 tanh(2 (R - r) / W) around the centre with the periodic (minimum-image)
    distance; cylinder=True measures r in the x-y plane only (a column along z)."""
    c = (nx / 2.0, ny / 2.0, nz / 2.0) if centre is None else centre
    d = []
    for n_, c_, shape in ((nx, c[0], (1, 1, nx)), (ny, c[1], (1, ny, 1)), (nz, c[2], (nz, 1, 1))):
        a = np.abs(np.arange(n_, dtype=np.float64) - c_)
        d.append(np.minimum(a, n_ - a).reshape(shape))
    r2 = d[0] ** 2 + d[1] ** 2 + (0.0 if cylinder else d[2] ** 2)
    r = np.sqrt(np.broadcast_to(r2, (nz, ny, nx)))
    return 0.5 + 0.5 * np.tanh(2.0 * (R - r) / W)


def layered_poiseuille3d(nxy=4, nz=100, mu_ratio=10.0, nu_B=0.1, G=1e-6, variant="qim",
                         visc="inverse_linear", sigma=0.001, M_phi=0.1, W=4.0, tau_h=1.0):
    """Layered Poiseuille flow (Sec. 4.3) in three dimensions: periodic in x and y, halfway
    bounce-back walls in z, body force G along x, fluid A on top, equal densities,
    mu_A/mu_B = mu_ratio; the channel coordinate z = k + 1/2 - nz/2 as in layered_phi."""
    mu_B = nu_B
    mu_A = mu_ratio * mu_B
    cfg = dict(BASE3D, name="layered_poiseuille3d", nx=nxy, ny=nxy, nz=nz, bc="walls_z",
               variant=variant, visc=visc, rho_A=1.0, rho_B=1.0, nu_A=mu_A, nu_B=nu_B,
               sigma=sigma, W=W, M_phi=M_phi, tau_h=tau_h, force_x=G, mu_A=mu_A, mu_B=mu_B)
    return cfg, plane_phi3d(nxy, nxy, nz, W, z0=nz / 2.0 - 0.5)


def table2_viscosities(mu_ratio, nu_mean=0.1):
    """Kinematic viscosities (nu_A, nu_B) for the layered channel at equal densities when only
    the ratio is given: the geometric mean is held at nu_mean, so both relaxation times stay
    moderate (at ratio 1000, tau = 10.0 and 0.509 instead of 300.5 and 0.8)."""
    r = float(mu_ratio) ** 0.5
    return nu_mean * r, nu_mean / r


def static_droplet3d(n=32, R=8.0, variant="qim", rho_ratio=10.0, sigma=0.01, tau=0.8,
                     tau_h=0.8, M_phi=0.02, W=4.0, cylinder=False):
    """Static droplet of phase A in an n^3 periodic box (the two-dimensional static-droplet
    parameters, F_s = -phi grad mu); cylinder=True gives a column of radius R along z."""
    cfg = dict(BASE3D, name="static_droplet3d", nx=n, ny=n, nz=n, variant=variant,
               fsurf="neg_phi_grad_mu", rho_A=rho_ratio, rho_B=1.0, nu_A=nu_from_tau(tau),
               nu_B=nu_from_tau(tau), sigma=sigma, W=W, M_phi=M_phi, tau_h=tau_h, R=R)
    return cfg, sphere_phi(n, n, n, R, W, cylinder=cylinder)


def plane_phi3d(nx, ny, nz, W, z0=None):
    """Flat interface normal to z at height z0 (equilibrium profile of eq. 9), A above."""
    z0 = nz / 2.0 if z0 is None else z0
    z = np.arange(nz, dtype=np.float64)[:, None, None] - z0
    return np.broadcast_to(0.5 + 0.5 * np.tanh(2.0 * z / W), (nz, ny, nx)).copy()
