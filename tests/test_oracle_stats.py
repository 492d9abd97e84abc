"""Pins of oracle/stats.py, the late-time statistic of the spinodal comparisons: the
characteristic length 2 pi / <k> of a single Fourier mode of wavenumber 2 pi m / n is n / m, in
any direction, whatever the amplitude, phase and mean; for two modes it is the power-weighted
harmonic combination."""
import numpy as np
import pytest

from oracle import stats


@pytest.mark.parametrize("m,axis", [(1, 0), (4, 1), (7, 0)])
def test_single_mode_length(m, axis):
    n = 64
    x = np.arange(n)
    wave = 0.3 * np.sin(2 * np.pi * m * x / n + 0.7) + 0.5
    phi = np.tile(wave[:, None] if axis == 0 else wave[None, :], (1, n) if axis == 0 else (n, 1))
    assert abs(stats.characteristic_length(phi) - n / m) < 1e-9 * n


def test_diagonal_mode_length():
    n = 64
    y, x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    phi = np.cos(2 * np.pi * (3 * x + 4 * y) / n)  # |k| = 2 pi 5 / n
    assert abs(stats.characteristic_length(phi) - n / 5) < 1e-9 * n


def test_two_modes_power_weighted():
    n = 128
    x = np.arange(n)
    a1, m1, a2, m2 = 1.0, 2, 0.5, 8
    row = a1 * np.sin(2 * np.pi * m1 * x / n) + a2 * np.cos(2 * np.pi * m2 * x / n)
    phi = np.tile(row[None, :], (n, 1))
    # S(k) holds a^2 at +-k for each mode: <k> = (a1^2 k1 + a2^2 k2) / (a1^2 + a2^2)
    k1, k2 = 2 * np.pi * m1 / n, 2 * np.pi * m2 / n
    kbar = (a1 ** 2 * k1 + a2 ** 2 * k2) / (a1 ** 2 + a2 ** 2)
    assert abs(stats.characteristic_length(phi) - 2 * np.pi / kbar) < 1e-9 * n
