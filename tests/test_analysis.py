"""The product's host analysis against single-mode closed forms and the oracle's
independent implementation."""
import numpy as np

from oracle import tfan_oracle as O
from paper_2511_00445_amd import analysis as A


def test_domain_length_single_modes_and_oracle():
    N = 128
    x = np.arange(N)[None, :] * np.ones((N, 1))
    y = x.T
    for n in (1, 4, 9):
        assert abs(A.domain_length(np.cos(2 * np.pi * n * y / N)) - N / n) < 1e-10
    rng = np.random.default_rng(3)
    phi = np.tanh(4 * rng.standard_normal((N, N)))
    assert abs(A.domain_length(phi) - O.domain_length(phi)) < 1e-10 * O.domain_length(phi)


def test_energy_spectrum_parseval_and_oracle():
    N = 64
    rng = np.random.default_rng(4)
    u = rng.standard_normal((2, N, N))
    E = A.energy_spectrum(u)
    assert abs(E.sum() - 0.5 * (u ** 2).sum(0).mean()) < 1e-12
    np.testing.assert_allclose(E, O.energy_spectrum(u), rtol=1e-12, atol=1e-16)
    assert len(A.band_average(E)) == 5
