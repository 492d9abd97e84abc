"""Statistics of a phase-separating field, for comparisons where pointwise parity no longer
applies (late-time spinodal decomposition is chaotic, Sec. 4.1).

TEST INFRASTRUCTURE: used by the tests and by the script that writes their golden values.

characteristic_length(phi): the domain size 2 pi / <k> with <k> the first moment of the
radially averaged structure factor S(k) = |FFT(phi - mean phi)|^2 over all nonzero
wavevectors of the periodic grid (wavenumbers 2 pi m / n). Plain numpy.
"""
import numpy as np


def structure_factor(phi):
    a = np.asarray(phi, dtype=np.float64)
    a = a - a.mean()
    S = np.abs(np.fft.fft2(a)) ** 2
    ky = 2.0 * np.pi * np.fft.fftfreq(a.shape[0])
    kx = 2.0 * np.pi * np.fft.fftfreq(a.shape[1])
    k = np.sqrt(ky[:, None] ** 2 + kx[None, :] ** 2)
    S[0, 0] = 0.0
    return k, S


def characteristic_length(phi):
    k, S = structure_factor(phi)
    return float(2.0 * np.pi * S.sum() / (k * S).sum())
