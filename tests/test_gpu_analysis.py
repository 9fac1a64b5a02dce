"""On-device observables (include/tfan_analysis.h) against the FP64 oracle
oracle/analysis_oracle.py on the same exported float32 states.

Tolerances: the spectra and correlations pass through a float32 FFT (relative
error ~ log2(n) x 6e-8 per coefficient) and are summed in float64, so shell values
agree to ~1e-6 of the largest; bounds 1e-5 relative (spectra, L) and 1e-5
absolute (correlations, which are normalised to 1 at r = 0).  Overlaps are float64
sums of float32 products: 1e-6.  Defect counts are integers decided in float32 on
both sides: exact.
"""
import sys

import numpy as np
import pytest

from oracle import analysis_oracle as A
from paper_2511_00445_amd.workloads import base_params, initial_fields

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def solver_state(n, steps, seed, zeta=0.02):
    import torch
    from paper_2511_00445_amd import Sim
    s = Sim(base_params(n, n, zeta=zeta))
    s.init_fields(**initial_fields(n, n, seed=seed, phi_noise=0.3, S0=0.2))
    s.step(steps)
    x = torch.empty((7, n, n), dtype=torch.float32, device="cuda")
    s.export_state(x)
    s.sync()
    return x


def compare(an, x, label):
    xh = x.cpu().numpy().astype(np.float64)
    sp, ref = an.spectra(x), A.spectra(xh)
    for k in ("E", "W", "S"):
        e = np.max(np.abs(sp[k] - ref[k])) / np.max(np.abs(ref[k]))
        assert e <= 1e-5, (label, k, e)
    np.testing.assert_array_equal(sp["count"], ref["count"])
    Lr = A.domain_length_from_spectrum(ref["S"], an.n)
    assert abs(sp["L"] - Lr) <= 1e-5 * Lr, (label, sp["L"], Lr)
    c, cr = an.correlations(x), A.correlations(xh)
    for k in ("uu", "ww", "QQ"):
        e = np.max(np.abs(c[k] - cr[k]))
        assert e <= 1e-5, (label, k, e)
    np.testing.assert_array_equal(c["count"], cr["count"])
    d, dr = an.defects(x), A.defects(xh)
    say(f"{label}: L {sp['L']:.4f} (oracle {Lr:.4f}); defects {d} (oracle {dr}); "
        f"C_uu(1) {c['uu'][1]:.5f} (oracle {cr['uu'][1]:.5f})")
    assert d == dr


@pytest.mark.parametrize("n,steps", [(8, 3), (64, 40), (256, 30)])
def test_observables_match_oracle(gpu, n, steps):
    from paper_2511_00445_amd import Analysis
    say(f"case: observables {n}x{n} after {steps} steps")
    an = Analysis(n)
    compare(an, solver_state(n, steps, seed=40 + n), f"{n}x{n}")


def test_observables_full_size_and_overlaps(gpu):
    import torch
    from paper_2511_00445_amd import Analysis
    say("case: observables 1024x1024, overlaps between two times")
    an = Analysis(1024)
    x0 = solver_state(1024, 20, seed=7)
    compare(an, x0, "1024x1024")
    x1 = solver_state(1024, 25, seed=7)
    o, orf = an.overlaps(x0, x1), A.temporal_overlaps(x0.cpu().numpy().astype(np.float64),
                                                      x1.cpu().numpy().astype(np.float64))
    assert np.max(np.abs(o - orf) / np.abs(orf)) <= 1e-6, (o, orf)
    o = an.overlaps(x0, x0)
    assert abs(o[0] - o[1]) <= 1e-12 * o[1] and abs(o[4] - o[5]) <= 1e-12 * o[5]


def test_constructed_fields(gpu):
    import torch
    from paper_2511_00445_amd import Analysis
    say("case: observables of constructed fields 64x64")
    n = 64
    an = Analysis(n)
    y, xg = np.mgrid[0:n, 0:n].astype(np.float64)
    x = np.zeros((7, n, n))
    th = 0.5 * np.arctan2(y - 31.5, xg - 15.5) - 0.5 * np.arctan2(y - 31.5, xg - 47.5)
    x[0] = 0.6 * np.cos(2 * np.pi * 4 * xg / n)
    x[1], x[2] = 0.2 * np.cos(2 * th), 0.2 * np.sin(2 * th)
    t = torch.tensor(x, dtype=torch.float32, device="cuda")
    assert an.defects(t) == (1, 1)
    sp = an.spectra(t)
    assert abs(sp["L"] - n / 4) <= 1e-5 * n / 4 and abs(sp["S"][4] - 0.18) <= 1e-6
    x[1], x[2] = 0.2, 0.0
    assert an.defects(torch.tensor(x, dtype=torch.float32, device="cuda")) == (0, 0)


def test_analysis_argument_errors(gpu):
    import torch
    import paper_2511_00445_amd as T
    say("case: analysis argument errors")
    for bad in (48, 4, 8192):
        with pytest.raises(T.TfanError):
            T.Analysis(bad)
    an = T.Analysis(16)
    with pytest.raises(T.TfanError):
        an.spectra(torch.zeros((7, 32, 32), device="cuda"))


def test_observables_maximum_size(gpu):
    """The largest grid the observables accept (4096 x 4096: 2,897 shells, 16.8 M
    plaquettes).  The state is taken after 300 steps, when the random initial
    director has relaxed: neighbouring angle differences near the +-pi/2 wrap
    (where a one-ulp difference between two float32 atan2 implementations could
    move a defect decision) are then confined to the defect cores."""
    from paper_2511_00445_amd import Analysis
    n = 4096
    say(f"case: observables {n}x{n} after 300 steps (maximum size)")
    an = Analysis(n)
    assert an.shells == 2897
    compare(an, solver_state(n, 300, seed=9), f"{n}x{n}")


@pytest.mark.parametrize("n,steps", [(64, 20), (512, 30)])
def test_all_in_one_call_equals_separate_calls(gpu, n, steps):
    """tfan_analysis_all shares the forward transforms: its results equal the
    separate calls bitwise, and the oracle to the bounds above."""
    from paper_2511_00445_amd import Analysis
    say(f"case: combined observables call {n}x{n}")
    an = Analysis(n)
    x = solver_state(n, steps, seed=60 + n)
    a, sp, c, d = an.all(x), an.spectra(x), an.correlations(x), an.defects(x)
    for k in ("E", "W", "S", "count"):
        np.testing.assert_array_equal(a[k], sp[k])
    assert a["L"] == sp["L"]
    for k in ("uu", "ww", "QQ"):
        np.testing.assert_array_equal(a[k], c[k])
    np.testing.assert_array_equal(a["count"], c["count"])
    assert a["defects"] == d
    ref = A.spectra(x.cpu().numpy().astype(np.float64))
    assert np.max(np.abs(a["E"] - ref["E"])) <= 1e-5 * np.max(np.abs(ref["E"]))
