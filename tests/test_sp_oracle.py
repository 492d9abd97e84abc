"""Pins of the FP64 CPU oracle of the generalized single-phase model with a mass source
(Sec. 2, Remarks 1 and 3): moment identities fixed by the lattice, exact global balances of
mass and momentum, the S = 0 limit (Guo et al. forced BGK) and the analytic steady flow driven
by a sinusoidal source, whose pressure carries the bulk viscosity set through Q."""
import math

import numpy as np
import pytest

from oracle import sp

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)
CS2 = 1.0 / 3.0
RNG = np.random.default_rng(5)


def moments(f):
    m0 = f.sum()
    m1 = np.array([(CX * f).sum(), (CY * f).sum()])
    m2 = np.array([[(CX * CX * f).sum(), (CX * CY * f).sum()], [(CY * CX * f).sum(), (CY * CY * f).sum()]])
    return m0, m1, m2


def test_equilibria_moments():
    for _ in range(5):
        rho, p, ux, uy = 1 + 0.1 * RNG.normal(), 0.01 * RNG.normal(), 0.05 * RNG.normal(), 0.05 * RNG.normal()
        u = np.array([ux, uy])
        # eq. (29bb): the moments of a nearly incompressible equilibrium
        m0, m1, m2 = moments(sp.equilibrium_ni(rho, ux, uy))
        assert abs(m0 - rho) < 1e-14
        np.testing.assert_allclose(m1, rho * u, atol=1e-15)
        np.testing.assert_allclose(m2, rho * CS2 * np.eye(2) + rho * np.outer(u, u), atol=1e-15)
        # eq. (25) with rho = 1: sum = rho_0, first moment u, second p I + uu
        m0, m1, m2 = moments(sp.equilibrium_inc(1.0, p, ux, uy))
        assert abs(m0 - 1.0) < 1e-14
        np.testing.assert_allclose(m1, u, atol=1e-15)
        np.testing.assert_allclose(m2, p * np.eye(2) + np.outer(u, u), atol=1e-15)


def test_force_term_moments():
    # eq. (27): sum G = S, sum c G = F, sum c c G = c_s^2 S I + A by the isotropy of the lattice
    for _ in range(5):
        S, Fx, Fy = RNG.normal(size=3) * 1e-3
        axx, axy, ayy = RNG.normal(size=3) * 1e-3
        m0, m1, m2 = moments(sp.force_distribution(S, Fx, Fy, axx, axy, ayy))
        assert abs(m0 - S) < 1e-18
        np.testing.assert_allclose(m1, [Fx, Fy], atol=1e-18)
        np.testing.assert_allclose(m2, CS2 * S * np.eye(2) + np.array([[axx, axy], [axy, ayy]]), atol=1e-18)


def test_pressure_inverts_incompressible_equilibrium():
    # eq. (28) applied to g^eq(p, u) with no source and no force returns p
    for _ in range(5):
        p, ux, uy = 0.01 * RNG.normal(), 0.05 * RNG.normal(), 0.05 * RNG.normal()
        g = sp.equilibrium_inc(1.0, p, ux, uy)
        assert abs(sp.pressure_inc(g, 0.0, ux, uy, 0.8, 0.0) - p) < 1e-16


def source_cfg(model, nx, ny, **kw):
    return dict(dict(nx=nx, ny=ny, model=model, nu=1.0 / 6.0, xi=0.0, full=True), **kw)


@pytest.mark.parametrize("model", ["nearly_incompressible", "incompressible"])
def test_global_mass_and_momentum_balance(model):
    # per step: total momentum sum(rho u) grows by sum F exactly (both models); in the nearly
    # incompressible model total rho~ = sum(g) + S/2 grows by sum S exactly (eq. 27aa)
    nx, ny = 12, 10
    S = 1e-3 * RNG.normal(size=(ny, nx)) + 2e-4
    Fx = 1e-4 * RNG.normal(size=(ny, nx)) + 1e-5
    Fy = 1e-4 * RNG.normal(size=(ny, nx))
    a0 = (1.0 + 1e-3 * RNG.normal(size=(ny, nx))) if model == "nearly_incompressible" else 1e-3 * RNG.normal(size=(ny, nx))
    o = sp.SpOracle(source_cfg(model, nx, ny)).init(a0, 1e-3 * RNG.normal(size=(ny, nx)),
                                                     1e-3 * RNG.normal(size=(ny, nx)), S, Fx, Fy)
    for _ in range(20):
        rho = o.read("rho")
        mom = np.array([(rho * o.read("ux")).sum(), (rho * o.read("uy")).sum()])
        m = o.sum_rho_tilde()
        o.step(1)
        rho = o.read("rho")
        mom2 = np.array([(rho * o.read("ux")).sum(), (rho * o.read("uy")).sum()])
        np.testing.assert_allclose(mom2 - mom, [Fx.sum(), Fy.sum()], rtol=1e-10, atol=1e-15)
        if model == "nearly_incompressible":
            assert abs(o.sum_rho_tilde() - m - S.sum()) < 1e-12


def poiseuille(model, ny, tau, G=1e-6):
    nu = (tau - 0.5) / 3.0
    cfg = dict(nx=3, ny=ny, model=model, nu=nu, bc="walls_y", full=True)
    o = sp.SpOracle(cfg).init(Fx=np.full((ny, 3), G))
    o.step(int(25 * ny * ny / nu / math.pi ** 2))
    u = o.read("ux")[:, 0]
    h = ny / 2.0
    y = np.arange(ny) + 0.5 - h
    ua = G / (2 * nu) * (h * h - y * y)
    return np.abs(u - ua).max() / ua.max()


@pytest.mark.parametrize("model", ["nearly_incompressible", "incompressible"])
def test_zero_source_limit_is_forced_bgk(model):
    # S = 0: both reductions are the forced BGK scheme of Guo et al.; with halfway bounce-back
    # the body-force channel flow is exact when (tau - 1/2)^2 = 3/16, second order otherwise
    assert poiseuille(model, 8, 0.5 + math.sqrt(3) / 4) < 1e-9
    e8, e16 = poiseuille(model, 8, 1.0), poiseuille(model, 16, 1.0)
    assert 3.5 < e8 / e16 < 4.5


def source_flow(model, nx, xi=0.0, S0=1e-4, full=True, steps=None):
    """Steady flow driven by S = S0 sin(kx) on a periodic nx x 3 grid. Continuity gives
    u_x = -(S0/k) cos(kx) (times 1/rho in the nearly incompressible model); the x momentum
    balance d_x(rho u^2 + p) = d_x((mu + xi) d_x u) gives the pressure up to a constant:
    p = -rho u^2 + (nu + xi) S0 sin(kx), i.e. a sin(kx) component of amplitude (nu + xi) S0."""
    ny = 3
    k = 2 * math.pi / nx
    x = np.arange(nx)
    S = np.tile(S0 * np.sin(k * x), (ny, 1))
    o = sp.SpOracle(source_cfg(model, nx, ny, xi=xi, full=full)).init(S=S)
    nu = 1.0 / 6.0
    o.step(steps or int(36 / ((nu + xi) * k * k)))  # ~36 slowest viscous e-folding times
    rho, u, p = o.read("rho")[1], o.read("ux")[1], o.read("p")[1]
    mass_flux = rho * u
    flux_err = np.abs(mass_flux - (-(S0 / k) * np.cos(k * x))).max() / (S0 / k)
    sin_amp = 2 * (p * np.sin(k * x)).mean()
    return flux_err, sin_amp, o


@pytest.mark.parametrize("model", ["nearly_incompressible", "incompressible"])
def test_source_flow_velocity_second_order(model):
    e16, _, _ = source_flow(model, 16)
    e32, _, _ = source_flow(model, 32)
    print(f"{model}: mass-flux error {e16:.3e} (nx 16), {e32:.3e} (nx 32)")
    assert e32 < 5e-3
    assert 3.0 < e16 / e32 < 5.0


@pytest.mark.parametrize("model", ["nearly_incompressible", "incompressible"])
@pytest.mark.parametrize("xi", [0.0, 0.1])
def test_source_flow_pressure_carries_bulk_viscosity(model, xi):
    # the sin(kx) part of the pressure is (nu + xi) S0: the bulk viscosity xi enters only
    # through Q of the force term, so this pins Q (div u) I of eq. (27)
    S0, nu = 1e-4, 1.0 / 6.0
    _, amp, _ = source_flow(model, 32, xi=xi, S0=S0)
    print(f"{model} xi {xi}: sin amplitude {amp:.6e} vs {(nu + xi) * S0:.6e}")
    assert abs(amp / ((nu + xi) * S0) - 1) < 0.02


def test_incompressible_remark_and_full_forms_agree_at_low_mach():
    # the terms Remark 3 drops (d_t p, grad p in F~, u u S) are higher order in Ma: at a small
    # source both forms give the same steady flow
    e_full, a_full, of = source_flow("incompressible", 32, full=True)
    e_rem, a_rem, orm = source_flow("incompressible", 32, full=False)
    np.testing.assert_allclose(of.read("ux"), orm.read("ux"), rtol=0, atol=1e-3 * 1e-4 * 32 / (2 * math.pi))
    assert abs(a_full / a_rem - 1) < 0.01


@pytest.mark.parametrize("tau", [0.8, 1.0, 1.5])
def test_incompressible_full_form_is_stable(tau):
    # d_t p taken at the current level (eq. 28 solved for p^n) keeps perturbations bounded; a
    # lagged difference p^{n-1} - p^{n-2} in the force term makes them grow by ~20% per step
    from paper_1902_08933_amd import workloads as W
    cfg, f = W.single_phase_source(20, 18, model="incompressible", S0=1e-4, F0=2e-6, seed=3,
                                   nu=(tau - 0.5) / 3.0, full=True)
    pert = 1e-10 * np.random.default_rng(0).normal(size=(18, 20))
    a = sp.SpOracle(cfg).init(f["a0"], f["ux"], f["uy"], f["S"], f["Fx"], f["Fy"]).step(400)
    b = sp.SpOracle(cfg).init(f["a0"] + pert, f["ux"], f["uy"], f["S"], f["Fx"], f["Fy"]).step(400)
    d = np.abs(a.read("p") - b.read("p")).max()
    print(f"tau {tau}: perturbation after 400 steps {d:.2e}")
    assert d < 1e-9


# ---- a force that depends on u, and Remark 4's explicit D_i G_i scheme -----------------------

def uniform_drag(scheme, lam, steps, u0=1e-3):
    nx = ny = 4
    cfg = dict(nx=nx, ny=ny, model="nearly_incompressible", nu=1.0 / 6.0, drag=lam, scheme=scheme)
    o = sp.SpOracle(cfg).init(ux=np.full((ny, nx), u0))
    us = []
    for _ in range(steps + 1):
        us.append(o.read("ux")[0, 0])
        o.step(1)
    return np.array(us)


def test_drag_time_discretizations_are_exact_recurrences():
    # uniform fluid under F = -lambda rho u: eq. (24) with the implicit velocity of eq. (27a)
    # advances the momentum by the trapezoidal rule, u_{n+1} = u_n (1 - lambda/2)/(1 + lambda/2);
    # Remark 4 by second-order Adams-Bashforth, m_{n+1} = m_n + (3 F_n - F_{n-1})/2 with
    # F_{-1} = F_0
    lam, n = 0.05, 60
    u = uniform_drag("eq24", lam, n)
    r = (1 - lam / 2) / (1 + lam / 2)
    np.testing.assert_allclose(u, u[0] * r ** np.arange(n + 1), rtol=1e-10)
    u = uniform_drag("remark4", lam, n)
    ref = [u[0], u[0] * (1 - lam)]
    for _ in range(n - 1):
        ref.append(ref[-1] - lam * (3 * ref[-1] - ref[-2]) / 2)
    np.testing.assert_allclose(u, np.array(ref), rtol=1e-10)  # round-off of 60 steps ~1e-12


@pytest.mark.parametrize("scheme", ["eq24", "remark4"])
def test_drag_decay_is_second_order_in_time(scheme):
    # at fixed time T = 2 / lambda_0 the error against exp(-lambda t) drops 4x when lambda halves
    def err(lam):
        n = int(round(2.0 / lam))
        u = uniform_drag(scheme, lam, n)
        return abs(u[-1] / u[0] - math.exp(-lam * n))
    e1, e2 = err(0.1), err(0.05)
    print(f"{scheme}: decay error {e1:.3e} (lambda 0.1), {e2:.3e} (0.05)")
    assert 3.5 < e1 / e2 < 4.5


def test_remark4_global_balances():
    # total rho~ grows by sum S per step; total momentum by (3 sum F_n - sum F_{n-1}) / 2, with
    # F = F_ext - lambda rho u evaluated on the state of each step
    nx, ny, lam = 12, 10, 0.02
    S = 1e-3 * RNG.normal(size=(ny, nx)) + 2e-4
    Fx = 1e-4 * RNG.normal(size=(ny, nx))
    Fy = 1e-4 * RNG.normal(size=(ny, nx))
    cfg = dict(nx=nx, ny=ny, model="nearly_incompressible", nu=0.1, drag=lam, scheme="remark4")
    o = sp.SpOracle(cfg).init(1 + 1e-3 * RNG.normal(size=(ny, nx)), 1e-3 * RNG.normal(size=(ny, nx)),
                              1e-3 * RNG.normal(size=(ny, nx)), S, Fx, Fy)

    def totals():
        rho, ux, uy = o.read("rho"), o.read("ux"), o.read("uy")
        F = np.array([(Fx - lam * rho * ux).sum(), (Fy - lam * rho * uy).sum()])
        return o.sum_rho_tilde(), np.array([(rho * ux).sum(), (rho * uy).sum()]), F
    m0, M0, F0 = totals()
    Fprev = F0
    for _ in range(15):
        o.step(1)
        m1, M1, F1 = totals()
        assert abs(m1 - m0 - S.sum()) < 1e-12
        np.testing.assert_allclose(M1 - M0, (3 * F0 - Fprev) / 2, rtol=1e-9, atol=1e-16)
        Fprev, m0, M0, F0 = F0, m1, M1, F1


def test_remark4_channel_flow_second_order():
    def channel(ny, G=1e-6, tau=1.0):
        nu = (tau - 0.5) / 3.0
        cfg = dict(nx=3, ny=ny, model="nearly_incompressible", nu=nu, bc="walls_y", scheme="remark4")
        o = sp.SpOracle(cfg).init(Fx=np.full((ny, 3), G))
        o.step(int(25 * ny * ny / nu / math.pi ** 2))
        u = o.read("ux")[:, 0]
        h = ny / 2.0
        y = np.arange(ny) + 0.5 - h
        ua = G / (2 * nu) * (h * h - y * y)
        return np.abs(u - ua).max() / ua.max()
    e8, e16 = channel(8), channel(16)
    print(f"Remark 4 channel: error {e8:.3e} (ny 8), {e16:.3e} (ny 16)")
    assert e16 < 2e-2
    assert 3.0 < e8 / e16 < 5.0
