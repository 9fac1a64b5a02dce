"""Pins of the observables oracle (oracle/analysis_oracle.py): closed forms of single
Fourier modes, Parseval, brute-force correlation sums, central-difference vorticity
of shear modes, constructed +-1/2 defects."""
import numpy as np

from oracle import analysis_oracle as A


def state(N, phi=None, qxx=None, qxy=None, ua=None, up=None):
    z = np.zeros((N, N))
    x = np.zeros((7, N, N))
    x[0] = np.ones((N, N)) if phi is None else phi
    x[1] = z if qxx is None else qxx
    x[2] = z if qxy is None else qxy
    if ua is not None:
        x[3:5] = ua
    if up is not None:
        x[5:7] = up
    return x


def test_shell_index_values():
    s = A.shell_index(16)
    assert s[4, 3] == 5 and s[1, 1] == 1 and s[2, 1] == 2 and s[2, 2] == 3 and s[0, 0] == 0
    assert s[8, 8] == 11 and s[-3, 4] == 5  # |(8, 8)| = 11.31; negative frequencies


def test_single_mode_spectra_and_length():
    N, n, a, b = 32, 3, 0.7, 0.4
    y = np.arange(N)[:, None] * np.ones((1, N))
    xg = np.ones((N, 1)) * np.arange(N)[None, :]
    u = np.stack([a * np.cos(2 * np.pi * n * y / N), np.zeros((N, N))])
    sp = A.spectra(state(N, ua=u))              # phi = 1: u_c = u_a
    assert abs(sp["E"][n] - a * a / 4) < 1e-14 and abs(sp["E"].sum() - a * a / 4) < 1e-14
    assert abs(sp["W"][n] - (2 * np.pi * n / N) ** 2 * a * a / 4) < 1e-14
    phi = b * np.cos(2 * np.pi * n * xg / N)
    sp = A.spectra(state(N, phi=phi))
    assert abs(sp["S"][n] - b * b / 2) < 1e-14
    assert abs(A.domain_length_from_spectrum(sp["S"], N) - N / n) < 1e-12
    assert sp["count"].sum() == N * N


def test_parseval_for_a_random_state():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(7, 16, 16)) * 0.1
    sp = A.spectra(x)
    u = A.mixed_velocity(x)
    assert abs(sp["E"].sum() - 0.5 * np.mean(np.sum(u * u, axis=0))) < 1e-14
    assert abs(sp["S"].sum() - np.mean(x[0] ** 2)) < 1e-14


def brute_radial(fields, N):
    """<sum_c f_c(x) f_c(x + r)> / <sum_c f_c^2> for every r by loops, then shell means."""
    norm = sum(np.mean(f * f) for f in fields)
    s = A.shell_index(N)
    acc = np.zeros(s.max() + 1)
    cnt = np.zeros(s.max() + 1)
    for ry in range(N):
        for rx in range(N):
            c = sum(np.mean(f * np.roll(np.roll(f, -ry, 0), -rx, 1)) for f in fields) / norm
            acc[s[ry, rx]] += c
            cnt[s[ry, rx]] += 1
    return acc / cnt


def test_correlations_against_brute_force():
    rng = np.random.default_rng(2)
    N = 8
    x = rng.normal(size=(7, N, N))
    x[0] = np.tanh(x[0])
    c = A.correlations(x)
    u = A.mixed_velocity(x)
    du = u - u.mean(axis=(1, 2), keepdims=True)
    w = A.vorticity(u)
    np.testing.assert_allclose(c["uu"], brute_radial([du[0], du[1]], N), atol=1e-12)
    np.testing.assert_allclose(c["ww"], brute_radial([w - w.mean()], N), atol=1e-12)
    np.testing.assert_allclose(c["QQ"], brute_radial([x[1], x[2]], N), atol=1e-12)
    assert c["uu"][0] == 1.0 or abs(c["uu"][0] - 1.0) < 1e-14


def test_vorticity_of_shear_modes():
    N, m = 32, 2
    y = np.arange(N)[:, None] * np.ones((1, N))
    xg = np.ones((N, 1)) * np.arange(N)[None, :]
    k = 2 * np.pi * m / N
    w = A.vorticity(np.stack([np.sin(k * y), np.zeros((N, N))]))
    np.testing.assert_allclose(w, -np.sin(k) * np.cos(k * y), atol=1e-14)
    w = A.vorticity(np.stack([np.zeros((N, N)), np.sin(k * xg)]))
    np.testing.assert_allclose(w, np.sin(k) * np.cos(k * xg), atol=1e-14)


def director_state(theta):
    N = theta.shape[0]
    return state(N, qxx=0.3 * np.cos(2 * theta), qxy=0.3 * np.sin(2 * theta))


def test_constructed_defects():
    N = 24
    y, x = np.mgrid[0:N, 0:N].astype(float)
    for q, want in ((0.5, (1, 0)), (-0.5, (0, 1))):
        th = q * np.arctan2(y - 11.5, x - 11.5)
        # far from the core the pattern is smooth except across the periodic seam, where
        # the winding of the whole box is exactly compensated; count inside the box only
        p, m = A.defects(director_state(th))
        assert (p >= want[0]) and (m >= want[1])
    th = np.full((N, N), 0.3)
    assert A.defects(director_state(th)) == (0, 0)
    # a +1/2, -1/2 pair on a periodic box: exactly one of each
    th = 0.5 * np.arctan2(y - 11.5, x - 5.5) - 0.5 * np.arctan2(y - 11.5, x - 17.5)
    assert A.defects(director_state(th)) == (1, 1)


def test_temporal_overlaps():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(7, 16, 16))
    o = A.temporal_overlaps(x, x)
    assert abs(o[0] - o[1]) < 1e-12 and abs(o[2] - o[3]) < 1e-12 and abs(o[4] - o[5]) < 1e-12
    y = x.copy()
    y[3:7] *= -1
    y[1:3] *= -1
    o = A.temporal_overlaps(x, y)
    assert abs(o[0] + o[1]) < 1e-12 and abs(o[2] + o[3]) < 1e-12 and abs(o[4] + o[5]) < 1e-12


def test_overlap_norms_closed_form():
    """Uniform fields: <|u_c|^2> = |u|^2, <Q:Q> = 2 S^2 for Q = S (cos 2t, sin 2t),
    and the vorticity of a uniform flow is zero."""
    N, S, t = 8, 0.3, 0.4
    u = np.stack([np.full((N, N), 0.02), np.full((N, N), -0.01)])
    x = state(N, qxx=np.full((N, N), S * np.cos(2 * t)), qxy=np.full((N, N), S * np.sin(2 * t)), ua=u)
    o = A.temporal_overlaps(x, x)
    assert abs(o[1] - (0.02 ** 2 + 0.01 ** 2)) < 1e-15 and abs(o[5] - 2 * S * S) < 1e-15 and o[3] == 0.0
