"""CPU check of the windowed oracle used by the full-size GPU parity tests."""
import numpy as np

from oracle.tfan_oracle import Oracle
from paper_2511_00445_amd.workloads import base_params, initial_fields
from tests.windows import window_oracle


def test_window_oracle_is_exact_inside():
    """CPU check of the windowed oracle used by the full-size parity tests."""
    p = base_params(64, 64, zeta=0.03, lam=1.5)
    ic = initial_fields(64, 64, seed=21, phi_noise=0.4, S0=0.3)
    full = Oracle(p)
    full.init_fields(**ic)
    full.step(2)
    ff = full.get_fields()
    wf, xs, ys = window_oracle(p, ic, 5, 33, 6, 2)
    for k in ("phi", "qxx", "qxy", "u_a"):
        np.testing.assert_allclose(wf[k], ff[k][..., ys[:, None], xs[None, :]], rtol=0, atol=1e-15)
