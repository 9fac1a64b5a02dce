"""Host analysis of solver snapshots (Results section observables).

- domain_length(phi): L = 2 pi sum_k Phi(k) / sum_k k Phi(k) from the structure factor,
  Phi the shell sum of |phi_hat|^2 over unit-width shells in n = k N / (2 pi), k = 0 excluded.
- energy_spectrum(u): E(n) = 1/2 sum over shell n of |u_hat|^2, u_hat = FFT(u) / N^2.
- band_average(E): octave bands [2^j, 2^(j+1)) of a shell spectrum.
Square periodic grids only.
"""
from __future__ import annotations

import numpy as np


def _shells(n: int) -> np.ndarray:
    """Shell number of every 2D FFT bin: |n| rounded to the nearest integer."""
    f = np.fft.fftfreq(n, d=1.0 / n)
    return np.rint(np.hypot(f[:, None], f[None, :])).astype(np.int64)


def _check_square(shape):
    if shape[-1] != shape[-2]:
        raise ValueError("square grids only")


def domain_length(phi: np.ndarray) -> float:
    _check_square(phi.shape)
    n = phi.shape[-1]
    power = np.abs(np.fft.fft2(phi)) ** 2  # normalisation cancels in the ratio
    sh = _shells(n)
    sums = np.zeros(sh.max() + 1)
    np.add.at(sums, sh.ravel(), power.ravel())
    idx = np.arange(sums.size)
    k = idx * (2.0 * np.pi / n)
    return float(2.0 * np.pi * sums[1:].sum() / (k[1:] * sums[1:]).sum())


def energy_spectrum(u: np.ndarray) -> np.ndarray:
    _check_square(u.shape)
    n = u.shape[-1]
    power = (np.abs(np.fft.fft2(u[0])) ** 2 + np.abs(np.fft.fft2(u[1])) ** 2) / float(n) ** 4
    sh = _shells(n)
    out = np.zeros(sh.max() + 1)
    np.add.at(out, sh.ravel(), 0.5 * power.ravel())
    return out


def band_average(E: np.ndarray, kmax: int | None = None) -> np.ndarray:
    """Sum of a shell spectrum over octave bands [1,2), [2,4), ... up to kmax."""
    kmax = kmax or (len(E) - 1)
    bands = []
    lo = 1
    while lo * 2 <= kmax + 1:
        bands.append(float(np.sum(E[lo:2 * lo])))
        lo *= 2
    return np.array(bands)


def mixture_velocity(phi: np.ndarray, u_a: np.ndarray, u_p: np.ndarray) -> np.ndarray:
    """u_c = c1 u_a + c2 u_p with c1 = (1 + phi)/2 (Results, barycentric velocity)."""
    c1 = 0.5 * (1.0 + phi)
    return c1 * u_a + (1.0 - c1) * u_p
