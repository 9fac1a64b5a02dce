"""P17: the plain-C oracle and the numpy oracle are two independent codings of the
same algorithm; they must agree to rounding on random states."""
import numpy as np
import pytest

from oracle.coracle import COracle
from oracle.tfan_oracle import Oracle
from paper_2511_00445_amd.workloads import base_params, initial_fields, random_velocity


@pytest.mark.parametrize("nx,ny,steps,over", [(16, 16, 5, {}), (24, 13, 4, dict(zeta=0.05, lam=2.0, gamma=0.4)),
                                              (64, 64, 3, dict(n_sub=3, tau_a=0.7, tau_p=1.4, A0=0.1,
                                                               gamma_ldg=5.0))])
def test_c_oracle_matches_numpy_oracle(nx, ny, steps, over):
    p = base_params(nx, ny, **over)
    ic = initial_fields(nx, ny, seed=17, phi_mean=0.1, phi_noise=0.5, S0=0.3)
    ua, up = random_velocity(nx, ny, 18, 5e-3), random_velocity(nx, ny, 19, 5e-3)
    a, b = Oracle(p), COracle(p)
    a.init_fields(**ic, u_a=ua, u_p=up)
    b.init_fields(**ic, u_a=ua, u_p=up)
    a.step(steps)
    b.step(steps)
    fa, fb = a.get_fields(), b.get_fields()
    for k in fa:
        scale = max(np.abs(fa[k]).max(), 1e-30)
        assert np.abs(fa[k] - fb[k]).max() <= 1e-12 * scale, (k, np.abs(fa[k] - fb[k]).max(), scale)


def test_c_oracle_results_do_not_depend_on_thread_count():
    """The thread count (set for the single-core CPU baseline) changes only the
    timing: every row is computed by one thread in a fixed order."""
    from oracle.coracle import set_threads, threads
    p = base_params(40, 24, zeta=0.02)
    ic = initial_fields(40, 24, seed=3, phi_noise=0.2, S0=0.2)
    out = []
    n = threads()
    try:
        for t in (1, max(n, 2)):
            set_threads(t)
            o = COracle(p)
            o.init_fields(ic["phi"], ic["qxx"], ic["qxy"])
            o.step(3)
            out.append(o.get_fields())
    finally:
        set_threads(n)
    for k in out[0]:
        np.testing.assert_array_equal(out[0][k], out[1][k])


def test_c_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    """The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
    host code only) runs the smallest grid, a ragged grid and a non-square one with
    no report: no out-of-bounds access in the periodic stencils, no leak."""
    import os
    import shutil
    import subprocess
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("gcc not available")
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "coracle_sanitize_main.c")
    exe = str(tmp_path / "coracle_sanitized")
    r = subprocess.run([cc, "-O1", "-g", "-std=c99", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        "-fno-omit-frame-pointer", src, "-o", exe, "-lm"], capture_output=True, text=True, timeout=300)
    if r.returncode != 0 and "asan" in r.stderr.lower():
        pytest.skip("no sanitizer runtime for gcc")
    assert r.returncode == 0, r.stderr[-2000:]
    for args in (("8", "8", "3", "5"), ("13", "9", "2", "1"), ("21", "34", "2", "4")):
        r = subprocess.run([exe, *args], capture_output=True, text=True, timeout=300)
        assert r.returncode == 0 and r.stdout.startswith("ok"), (args, r.stdout, r.stderr[-3000:])
