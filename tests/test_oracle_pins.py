"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test checks an oracle function against an independent property: a moment identity the
paper's Chapman-Enskog analysis requires (Appendix A), a closed form (Fourier symbols of the
stencils, the tanh profile that zeroes the chemical potential), an inverse relation, or a
derivation the paper prints (Appendix B). None of them re-types the formula under test.

The D2Q9 lattice below is transcribed from the velocity matrix printed in Sec. 2.2 (after
eq. 25); it is the test's own copy, so an ordering or sign error in the oracle's table breaks
the moment identities.
"""
import math

import numpy as np
import pytest

import oracle

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
CS2 = 1.0 / 3.0
RNG = np.random.default_rng(12345)


def moments(f):
    m0 = f.sum()
    m1 = np.array([(CX * f).sum(), (CY * f).sum()])
    m2 = np.array([[(CX * CX * f).sum(), (CX * CY * f).sum()],
                   [(CY * CX * f).sum(), (CY * CY * f).sum()]])
    return m0, m1, m2


def test_lattice_isotropy_of_transcription():
    # sanity of the test's own lattice: sum w = 1, sum w c = 0, sum w c c = c_s^2 I
    assert abs(W.sum() - 1) < 1e-15
    assert abs((W * CX).sum()) < 1e-15 and abs((W * CY).sum()) < 1e-15
    assert abs((W * CX * CX).sum() - CS2) < 1e-15 and abs((W * CX * CY).sum()) < 1e-15


@pytest.mark.parametrize("trial", range(20))
def test_equilibrium_g_moments(trial):
    # Appendix A, eq. (a23) and the line after it: M0 = rho~ (= rho_0 = 1 in the two-phase
    # model), M1 = rho u, M2 = p I + rho u u
    p, rho = RNG.normal() * 1e-2, 0.5 + 5 * RNG.random()
    ux, uy = RNG.normal(size=2) * 0.05
    geq = oracle.equilibrium_g(p, rho, ux, uy)
    m0, m1, m2 = moments(geq)
    assert abs(m0 - 1.0) < 1e-14
    np.testing.assert_allclose(m1, rho * np.array([ux, uy]), atol=1e-15, rtol=1e-13)
    expect = p * np.eye(2) + rho * np.outer([ux, uy], [ux, uy])
    np.testing.assert_allclose(m2, expect, atol=1e-15, rtol=1e-13)


def test_pressure_inverts_equilibrium():
    # eq. (28) applied to an equilibrium state with S = 0, G_0 = 0 returns the pressure
    # the equilibrium was built from (sum_{i!=0} g_i^eq = p (1-w0)/c_s^2 - rho s_0(u))
    for _ in range(20):
        p, rho = RNG.normal() * 1e-2, 0.5 + 5 * RNG.random()
        ux, uy = RNG.normal(size=2) * 0.05
        geq = oracle.equilibrium_g(p, rho, ux, uy)
        got = oracle.pressure(geq, 0.0, rho, ux, uy, 0.8, 0.0, True)
        assert abs(got - p) < 1e-15 + 1e-12 * abs(p)


def test_pressure_matches_appendix_b_derivation():
    # Appendix B: when sum_i g_i + S/2 = rho~ (eq. a14 with sum G = S), eq. (28) equals the
    # first line of the derivation, c_s^2/(1-w0) [rho~ + rho s_0(u) - g_0 + (tau-1/2) G_0],
    # which uses g_0 where eq. (28) does not.
    for _ in range(20):
        g = RNG.normal(size=9) * 1e-3
        S = RNG.normal() * 1e-4
        g[0] = 1.0 - S / 2 - g[1:].sum()
        rho, tau, G0 = 1 + RNG.random(), 0.6 + RNG.random(), RNG.normal() * 1e-5
        ux, uy = RNG.normal(size=2) * 0.05
        s0 = W[0] * (-(ux * ux + uy * uy) / (2 * CS2))
        expect = CS2 / (1 - W[0]) * (1.0 + rho * s0 - g[0] + (tau - 0.5) * G0)
        got = oracle.pressure(g, S, rho, ux, uy, tau, G0, True)
        assert abs(got - expect) < 1e-14


def _random_force_inputs():
    rho = 0.5 + 5 * RNG.random()
    ux, uy = RNG.normal(size=2) * 0.05
    Fx, Fy = RNG.normal(size=2) * 1e-4
    gpx, gpy = RNG.normal(size=2) * 1e-4
    grx, gry = RNG.normal(size=2) * 1e-2
    S1 = RNG.normal() * 1e-4
    S = ux * grx + uy * gry + rho * S1          # Sec. 3.1
    Ftx, Fty = Fx - gpx + CS2 * grx, Fy - gpy + CS2 * gry   # F~ = F - grad(p - rho c_s^2)
    return rho, ux, uy, Fx, Fy, gpx, gpy, Ftx, Fty, S, S1


@pytest.mark.parametrize("trial", range(20))
def test_force_distribution_moments(trial):
    # eq. (a23): sum G = S; eq. (a25aa): sum c G = F; and by lattice isotropy the second moment
    # of eq. (34) is c_s^2 S I + A with A = u F~ + F~ u + (2/d) rho c_s^2 S1 I
    rho, ux, uy, Fx, Fy, gpx, gpy, Ftx, Fty, S, S1 = _random_force_inputs()
    G = oracle.force_distribution(rho, ux, uy, Fx, Fy, Ftx, Fty, S, S1)
    m0, m1, m2 = moments(G)
    assert abs(m0 - S) < 1e-18 + 1e-13 * abs(S)
    np.testing.assert_allclose(m1, [Fx, Fy], atol=1e-18, rtol=1e-12)
    u, Ft = np.array([ux, uy]), np.array([Ftx, Fty])
    A = np.outer(u, Ft) + np.outer(Ft, u) + rho * CS2 * S1 * np.eye(2)
    np.testing.assert_allclose(m2, CS2 * S * np.eye(2) + A, atol=1e-18, rtol=1e-11)


def test_force_distribution_rest_component_closed_form():
    # eq. (34) at i = 0 with S = u.grad(rho) + rho S1 and F~ = F - grad p + c_s^2 grad(rho):
    # the rho S1 terms cancel (tr I = d) and G_0 = -(w0 / c_s^2) u.(F - grad p)
    for _ in range(20):
        rho, ux, uy, Fx, Fy, gpx, gpy, Ftx, Fty, S, S1 = _random_force_inputs()
        G = oracle.force_distribution(rho, ux, uy, Fx, Fy, Ftx, Fty, S, S1)
        expect = -(W[0] / CS2) * (ux * (Fx - gpx) + uy * (Fy - gpy))
        assert abs(G[0] - expect) < 1e-19 + 1e-11 * abs(expect)


def test_simplified_G0_differs_by_lost_trace():
    # the simplified G_0 printed after eq. (34) evaluates (2/d) rho c_s^2 S1 I : I as
    # (2/d) rho c_s^2 S1 instead of 2 rho c_s^2 S1; the difference is w0 (1 - 1/d) rho S1,
    # and it coincides with eq. (34) when S1 = 0
    for _ in range(20):
        rho, ux, uy, Fx, Fy, gpx, gpy, Ftx, Fty, S, S1 = _random_force_inputs()
        G = oracle.force_distribution(rho, ux, uy, Fx, Fy, Ftx, Fty, S, S1)
        gB = oracle.G0_simplified(rho, ux, uy, Fx, Fy, gpx, gpy, S1)
        assert abs((gB - G[0]) - W[0] * 0.5 * rho * S1) < 1e-19 + 1e-11 * abs(rho * S1)
        gB0 = oracle.G0_simplified(rho, ux, uy, Fx, Fy, gpx, gpy, 0.0)
        G0 = oracle.force_distribution(rho, ux, uy, Fx, Fy, Ftx, Fty, S - rho * S1, 0.0)[0]
        assert abs(gB0 - G0) < 1e-19 + 1e-11 * abs(G0)


def test_pressure_eq28_equals_eq28aa():
    # eq. (28) and eq. (28aa) agree because sum_i G_i = S
    for _ in range(20):
        rho, ux, uy, Fx, Fy, gpx, gpy, Ftx, Fty, S, S1 = _random_force_inputs()
        G = oracle.force_distribution(rho, ux, uy, Fx, Fy, Ftx, Fty, S, S1)
        g = RNG.normal(size=9) * 1e-3
        tau = 0.6 + RNG.random()
        a = oracle.pressure(g, S, rho, ux, uy, tau, G[0], True)
        b = oracle.pressure(g, S, rho, ux, uy, tau, S - G[1:].sum(), True)
        assert abs(a - b) < 1e-17
        c = oracle.pressure(g, S, rho, ux, uy, tau, G[0], False)  # eq. (29)
        assert abs((a - c) - CS2 / (1 - W[0]) * (tau - 0.5) * G[0]) < 1e-17


@pytest.mark.parametrize("trial", range(10))
def test_equilibrium_h_and_source_moments(trial):
    # eq. (11): sum h^eq = phi, sum c h^eq = phi u, sum c c h^eq = eta mu c_s^2 I
    phi, mu, eta = RNG.random(), RNG.normal() * 1e-3, 0.1 + RNG.random()
    ux, uy = RNG.normal(size=2) * 0.05
    heq = oracle.equilibrium_h(phi, mu, eta, ux, uy)
    m0, m1, m2 = moments(heq)
    assert abs(m0 - phi) < 1e-15
    np.testing.assert_allclose(m1, [phi * ux, phi * uy], atol=1e-16, rtol=1e-13)
    np.testing.assert_allclose(m2, eta * mu * CS2 * np.eye(2), atol=1e-17, rtol=1e-12)
    # eq. (14) with the first-order difference: sum R = 0, sum c R = (1 - 1/2tau) d(phi u)
    tau = 0.6 + RNG.random()
    a = RNG.normal(size=4) * 1e-3
    R = oracle.source_R(tau, *a)
    m0, m1, _ = moments(R)
    assert abs(m0) < 1e-18
    np.testing.assert_allclose(m1, (1 - 0.5 / tau) * np.array([a[0] - a[2], a[1] - a[3]]),
                               atol=1e-18, rtol=1e-12)


def test_free_energy_coefficients():
    # eqs. (6)-(7) used forward: W = sqrt(8 kappa / beta), sigma = sqrt(2 kappa beta) / 6
    for sigma, Wd in [(0.01, 4.0), (0.001, 4.0), (0.03, 5.0)]:
        beta, kappa = oracle.free_energy_coeffs(sigma, Wd)
        assert abs(math.sqrt(8 * kappa / beta) - Wd) < 1e-12
        assert abs(math.sqrt(2 * kappa * beta) / 6 - sigma) < 1e-15


def test_plane_profile_zeroes_chemical_potential():
    # eq. (9) minimises the free energy: mu of eq. (8) vanishes on phi = 1/2 + 1/2 tanh(2z/W)
    # when lap(phi) is the exact second derivative of the profile
    sigma, Wd = 0.01, 4.0
    beta, kappa = oracle.free_energy_coeffs(sigma, Wd)
    for z in np.linspace(-8, 8, 33):
        t = math.tanh(2 * z / Wd)
        phi = 0.5 + 0.5 * t
        d2 = -(4.0 / Wd ** 2) * t * (1 - t * t)  # d^2/dz^2 of 1/2 tanh(2z/W)
        assert abs(oracle.chemical_potential(beta, kappa, phi, d2)) < 1e-16


def test_mobility_and_gamma():
    # eq. (17) forward: M = eta c_s^2 (tau_h - 1/2)
    for M, tau in [(0.02, 0.8), (0.1, 1.0), (6.667, 1.0)]:
        assert abs(oracle.eta(M, tau) * CS2 * (tau - 0.5) - M) < 1e-14
    # Sec. 3.2.1: with rho linear in phi (eq. 3aa), mass conservation and eq. (30) give
    # rho_B div(u) = -(rho_A - rho_B) div(M grad mu), i.e. gamma rho_B = rho_A - rho_B
    for ra, rb in [(10, 1), (1, 1e-3), (3, 1), (1, 1)]:
        assert abs(oracle.gamma(ra, rb) * rb - (ra - rb)) < 1e-12


def test_density_and_viscosity_closures():
    cfg = dict(rho_A=10.0, rho_B=2.0, nu_A=0.05, nu_B=0.2, sigma=0.01, W=4, M_phi=0.1,
               tau_h=1.0)
    # eq. (3aa): rho(phi_A = 1) = rho_A, rho(phi_B = 0) = rho_B, linear in between
    assert oracle.density(cfg, 1.0) == 10.0 and oracle.density(cfg, 0.0) == 2.0
    assert abs(oracle.density(cfg, 0.25) - 4.0) < 1e-15
    # inverse-linear viscosity: 1/nu linear in phi between 1/nu_B and 1/nu_A
    assert abs(oracle.viscosity(cfg, 1.0) - 0.05) < 1e-15
    assert abs(oracle.viscosity(cfg, 0.0) - 0.2) < 1e-15
    assert abs(1 / oracle.viscosity(cfg, 0.5) - 0.5 * (20 + 5)) < 1e-12
    # step form of Sec. 4.3: dynamic viscosity rho nu jumps at phi = 1/2
    cs = dict(cfg, visc="step")
    assert abs(oracle.viscosity(cs, 0.6) * oracle.density(cs, 0.6) - 10 * 0.05) < 1e-15
    assert abs(oracle.viscosity(cs, 0.4) * oracle.density(cs, 0.4) - 2 * 0.2) < 1e-15
    # clamping keeps rho and nu within the two phases
    cc = dict(cfg, clamp_props=True)
    assert oracle.density(cc, 1.2) == 10.0 and oracle.density(cc, -0.1) == 2.0


@pytest.mark.parametrize("kx,ky", [(1, 0), (0, 2), (3, 1), (5, 7), (16, 3)])
def test_stencil_fourier_symbols(kx, ky):
    # eq. (30a) and eq. (30b) on a plane wave: grad_x sin(k.x) = sin(kx)(2 + cos ky)/3 cos(k.x),
    # lap sin(k.x) = (8 cos kx + 8 cos ky + 4 cos kx cos ky - 20)/6 sin(k.x)
    N = 32
    ax, ay = 2 * np.pi * kx / N, 2 * np.pi * ky / N
    x = np.arange(N)[None, :]
    y = np.arange(N)[:, None]
    z = np.sin(ax * x + ay * y)
    c = np.cos(ax * x + ay * y)
    gx, gy = oracle.gradient(z)
    lap = oracle.laplacian(z)
    np.testing.assert_allclose(gx, np.sin(ax) * (2 + np.cos(ay)) / 3 * c, atol=1e-13)
    np.testing.assert_allclose(gy, np.sin(ay) * (2 + np.cos(ax)) / 3 * c, atol=1e-13)
    sym = (8 * np.cos(ax) + 8 * np.cos(ay) + 4 * np.cos(ax) * np.cos(ay) - 20) / 6
    np.testing.assert_allclose(lap, sym * z, atol=1e-13)


def test_stencil_wall_mirror_is_even_extension():
    # with walls, the ghost row is the mirror image about the wall half a cell away, so a field
    # even about both walls, cos(pi m (j + 1/2) / ny), has the same symbol as on a periodic grid
    nx, ny, m, kx = 16, 12, 3, 2
    ax, ay = 2 * np.pi * kx / nx, np.pi * m / ny
    x = np.arange(nx)[None, :]
    y = np.arange(ny)[:, None] + 0.5
    z = np.cos(ax * x) * np.cos(ay * y)
    lap = oracle.laplacian(z, bc="walls_y")
    sym = (8 * np.cos(ax) + 8 * np.cos(ay) + 4 * np.cos(ax) * np.cos(ay) - 20) / 6
    np.testing.assert_allclose(lap, sym * z, atol=1e-13)
    gx, gy = oracle.gradient(z, bc="walls_y")
    np.testing.assert_allclose(gy, -np.sin(ay) * (2 + np.cos(ax)) / 3 * np.cos(ax * x) * np.sin(ay * y),
                               atol=1e-13)
