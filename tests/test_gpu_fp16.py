"""Populations stored as binary16 (float32 arithmetic): errors against the FP64 oracle,
conservation and checkpoints.

Stated tolerances.  Each step rounds every stored population deviation f - w_i rho0 to
binary16 (unit roundoff u16 = 2^-11 = 4.9e-4).  On the 64x64 workload after 100-200
steps this was measured at: phi 6e-6-8e-6, Q 1.1e-4-1.7e-4, u_a 1.0e-3-1.3e-3,
u_p 5.8e-3, rho_a - 1 5e-4-1e-3 (relative L2; the float32 path is at <= 3e-6).
The passive fluid is driven only by drag and the c2 share of the capillary force, so
its velocity is small and carries the largest relative error.  Bounds below are those
values with a margin of about 4x.
"""
import sys

import numpy as np
import pytest

from oracle.coracle import COracle
from paper_2511_00445_amd.workloads import base_params, initial_fields, workload_params

pytestmark = pytest.mark.gpu
BOUNDS = {"phi": 5e-5, "qxx": 1e-3, "qxy": 1e-3, "u_a": 5e-3, "u_p": 2.5e-2}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("steps", [100, 200])
def test_fp16_storage_error_against_oracle(gpu, steps):
    from paper_2511_00445_amd import Sim
    say(f"case: fp16 storage 64x64, {steps} steps")
    p = workload_params("small_64")
    ic = initial_fields(64, 64, seed=0)
    o = COracle(p)
    o.init_fields(**ic)
    o.step(steps)
    of = o.get_fields()
    s = Sim(dict(p, storage=1))
    s.init_fields(**ic)
    s.step(steps)
    g = s.get_fields()
    errs = {k: rel(g[k], of[k]) for k in BOUNDS}
    errs["rho_a"] = rel(g["rho_a"] - 1, of["rho_a"] - 1)
    say(f"fp16 relative L2 after {steps} steps: {errs}")
    for k, b in BOUNDS.items():
        assert errs[k] <= b, (k, errs[k], b)
    assert errs["rho_a"] <= 5e-3


def test_fp16_storage_ragged_grid(gpu):
    from paper_2511_00445_amd import Sim
    say("case: fp16 ragged 50x37")
    p = base_params(50, 37, zeta=0.02, gamma=0.2, lam=0.9, tau_a=0.8, tau_p=1.3)
    ic = initial_fields(50, 37, seed=1, phi_mean=0.1, phi_noise=0.3, S0=0.2)
    o = COracle(p)
    o.init_fields(**ic)
    o.step(25)
    of = o.get_fields()
    s = Sim(dict(p, storage=1))
    s.init_fields(**ic)
    s.step(25)
    g = s.get_fields()
    for k in ("phi", "qxx", "qxy", "u_a"):
        assert rel(g[k], of[k]) <= BOUNDS[k], (k, rel(g[k], of[k]))


def test_fp16_storage_conservation_and_checkpoint(gpu):
    from paper_2511_00445_amd import Sim
    say("case: fp16 conservation and checkpoint")
    p = dict(workload_params("small_64", zeta=0.02), storage=1)
    ic = initial_fields(64, 64, seed=5, phi_mean=0.3, phi_noise=0.3)
    s = Sim(p)
    s.init_fields(**ic)
    d0 = s.diagnostics()
    s.step(1000)
    d1 = s.diagnostics()
    mass_drift = abs(d1["mass_a"] - d0["mass_a"]) / d0["mass_a"]
    phi_drift = abs(d1["phi_sum"] - d0["phi_sum"]) / np.abs(ic["phi"]).sum()
    say(f"fp16: per-fluid mass drift {mass_drift:.3e}, phi mass drift {phi_drift:.3e} after 1000 steps")
    assert d1["status"] == 0 and mass_drift < 1e-4 and phi_drift < 1e-5
    ck = s.get_state()
    assert ck.size == 8 + 64 * 64 * (18 * 2 + 3 * 4)
    s.step(10)
    ref = s.get_state()
    s.set_state(ck)
    s.step(10)
    assert np.array_equal(s.get_state(), ref)
