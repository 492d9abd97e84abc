"""Closed-form solutions used as expected values by the tests (not inputs, not the method)."""
import numpy as np


def layered_analytic_ux(ny, G, mu_A, mu_B):
    """Steady layered-Poiseuille velocity, eq. (37), at the node rows of the layered order
    parameter (cell-centred rows y = j + 1/2 - ny/2, phase A above y = 0, halfway walls)."""
    h = ny / 2.0
    y = np.arange(ny, dtype=np.float64) + 0.5 - h
    s = y / h
    k = (mu_A - mu_B) / (mu_A + mu_B)
    top = G * h * h / (2 * mu_A) * (-s * s - s * k + 2 * mu_A / (mu_A + mu_B))
    bot = G * h * h / (2 * mu_B) * (-s * s - s * k + 2 * mu_B / (mu_A + mu_B))
    return np.where(y > 0, top, bot)
