"""FP64 CPU oracle of the Results-section observables (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU baseline may import this
module; the product path never does.

Inputs are solver states as exported by the library: [7][N][N] float arrays
(phi, Qxx, Qxy, u_a,x, u_a,y, u_p,x, u_p,y) on a square periodic grid.
Definitions (Results section), each written out plainly with numpy's FFT as the
only library step:

- mixed velocity u_c = c1 u_a + c2 u_p, c1 = (1 + phi)/2, c2 = 1 - c1; mixed
  vorticity omega_c = d_x u_c,y - d_y u_c,x with central differences;
- hat f = FFT(f) / N^2; wavevector index n = (n_x, n_y) in (-N/2, N/2]; shell of n
  = the integer nearest to |n|;
- kinetic-energy spectrum E(s) = 1/2 sum over shell s of |hat u_c|^2; enstrophy
  spectrum W(s) = k_s^2 E(s) with k_s = 2 pi s / N; phase-field spectrum
  S(s) = sum over shell s of |hat phi|^2;
- domain length L = 2 pi sum_{s>0} S(s) / sum_{s>0} k_s S(s);
- spatial correlations: C(r) = <f(x) . f(x + r)> / <f . f> for f = delta u_c
  (fluctuation about the mean), delta omega_c and Q (with Q : Q' =
  2 (Qxx Qxx' + Qxy Qxy')), evaluated for every displacement r on the periodic
  grid and averaged over displacement shells (integer nearest to |r|, minimum
  image);
- temporal correlation numerators and norms between two states:
  <u_c . u_c'>, <|u_c|^2>, <omega_c omega_c'>, <omega_c^2>, <Q : Q'>, <Q : Q>;
- +-1/2 defects by winding number: director angle theta = atan2(Qxy, Qxx) / 2
  (Q = S (cos 2 theta, sin 2 theta)); around every elementary plaquette
  (x, y) -> (x+1, y) -> (x+1, y+1) -> (x, y+1) -> (x, y) the angle differences are
  wrapped into [-pi/2, pi/2) and summed; a sum of +pi (-pi) is a +1/2 (-1/2)
  defect.  The angle and wrap decisions are taken in float32, the precision of
  the exported state.
"""
from __future__ import annotations

import numpy as np


def mixed_velocity(x):
    c1 = 0.5 * (1.0 + x[0])
    return np.stack([c1 * x[3] + (1.0 - c1) * x[5], c1 * x[4] + (1.0 - c1) * x[6]])


def central_dx(f):
    return 0.5 * (np.roll(f, -1, axis=-1) - np.roll(f, 1, axis=-1))


def central_dy(f):
    return 0.5 * (np.roll(f, -1, axis=-2) - np.roll(f, 1, axis=-2))


def vorticity(u):
    return central_dx(u[1]) - central_dy(u[0])


def shell_index(N):
    """Shell (nearest integer to |n|) of every FFT bin and of every displacement."""
    f = np.fft.fftfreq(N, d=1.0 / N)
    n2 = f[:, None] ** 2 + f[None, :] ** 2
    s = np.floor(np.sqrt(n2)).astype(np.int64)
    s += ((s + 0.5) ** 2 <= n2).astype(np.int64)   # nearest integer to sqrt(n2)
    return s


def shell_sum(values, N):
    s = shell_index(N)
    out = np.zeros(s.max() + 1)
    np.add.at(out, s.ravel(), values.ravel())
    return out


def shell_counts(N):
    s = shell_index(N)
    return np.bincount(s.ravel()).astype(np.float64)


def hat(f):
    return np.fft.fft2(f) / float(f.shape[-1]) ** 2


def spectra(x):
    """E(s), W(s), S(s) and the shell counts of a state [7][N][N]."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[-1]
    u = mixed_velocity(x)
    E = 0.5 * shell_sum(np.abs(hat(u[0])) ** 2 + np.abs(hat(u[1])) ** 2, N)
    S = shell_sum(np.abs(hat(x[0])) ** 2, N)
    k = 2.0 * np.pi * np.arange(E.size) / N
    return dict(E=E, W=k ** 2 * E, S=S, count=shell_counts(N))


def domain_length_from_spectrum(S, N):
    k = 2.0 * np.pi * np.arange(S.size) / N
    return float(2.0 * np.pi * S[1:].sum() / (k[1:] * S[1:]).sum())


def _autocorrelation(fields):
    """sum over components of <f(x) f(x + r)> for every displacement r (circular)."""
    acc = 0.0
    for f in fields:
        F = np.fft.fft2(f)
        acc = acc + np.real(np.fft.ifft2(np.abs(F) ** 2)) / f.size
    return acc


def correlations(x):
    """Radially averaged Cuu(r), Cww(r), CQQ(r) and the shell counts."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[-1]
    u = mixed_velocity(x)
    du = u - u.mean(axis=(1, 2), keepdims=True)
    w = vorticity(u)
    dw = w - w.mean()
    cnt = shell_counts(N)
    out = {}
    for name, comps in (("uu", [du[0], du[1]]), ("ww", [dw]), ("QQ", [x[1], x[2]])):
        c = _autocorrelation(comps)
        out[name] = shell_sum(c / c[0, 0], N) / cnt
    out["count"] = cnt
    return out


def temporal_overlaps(x0, x1):
    """<u_c.u_c'>, <|u_c|^2>, <w w'>, <w^2>, <Q:Q'>, <Q:Q> between states x0 and x1."""
    a, b = np.asarray(x0, dtype=np.float64), np.asarray(x1, dtype=np.float64)
    ua, ub = mixed_velocity(a), mixed_velocity(b)
    wa, wb = vorticity(ua), vorticity(ub)
    return np.array([np.mean(np.sum(ua * ub, axis=0)), np.mean(np.sum(ua * ua, axis=0)),
                     np.mean(wa * wb), np.mean(wa * wa),
                     np.mean(2.0 * (a[1] * b[1] + a[2] * b[2])), np.mean(2.0 * (a[1] ** 2 + a[2] ** 2))])


def defects(x):
    """(number of +1/2, number of -1/2 defects) by winding number (float32 decisions)."""
    qxx = np.asarray(x[1], dtype=np.float32)
    qxy = np.asarray(x[2], dtype=np.float32)
    th = np.float32(0.5) * np.arctan2(qxy, qxx)
    half_pi = np.float32(np.pi / 2)

    def wrap(d):
        # into [-pi/2, pi/2)
        d = np.where(d >= half_pi, d - np.float32(np.pi), d)
        return np.where(d < -half_pi, d + np.float32(np.pi), d)

    t00 = th
    t10 = np.roll(th, -1, axis=1)                  # (x+1, y)
    t11 = np.roll(np.roll(th, -1, axis=1), -1, axis=0)
    t01 = np.roll(th, -1, axis=0)                  # (x, y+1)
    s = wrap(t10 - t00) + wrap(t11 - t10) + wrap(t01 - t11) + wrap(t00 - t01)
    plus = int(np.count_nonzero(s > half_pi))
    minus = int(np.count_nonzero(s < -half_pi))
    return plus, minus
