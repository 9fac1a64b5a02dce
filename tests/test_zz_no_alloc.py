"""tfan_analysis_overlaps_noalloc (the allocation-free variant of
tfan_analysis_overlaps) against the handle-based entry point, through the C ABI:
two calls in a row on the same GPU, the second on a smaller grid, each equal bit
for bit to the handle-based call (the same kernels reduce in the same order), and
the size checks."""
import ctypes
import sys

import numpy as np
import pytest

from paper_2511_00445_amd.workloads import base_params, initial_fields

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _states(n, seed):
    import torch
    from paper_2511_00445_amd import Sim
    p = base_params(n, n, zeta=0.02)
    s = Sim(p)
    s.init_fields(**initial_fields(n, n, seed=seed, phi_noise=0.3, S0=0.2))
    a = torch.empty((7, n, n), dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    s.step(3)
    s.export_state(a)
    s.step(4)
    s.export_state(b)
    s.sync()
    s.close()
    return a, b


def test_overlaps_noalloc_matches_handle_call(gpu):
    import torch
    from paper_2511_00445_amd import Analysis, TFAN_EINVAL, TfanError
    from paper_2511_00445_amd.binding import analysis_overlaps_noalloc, load_library
    lib = load_library()
    for n, seed in ((64, 41), (32, 42)):
        say(f"case: overlaps without allocation, {n}x{n}, seed {seed}")
        a, b = _states(n, seed)
        an = Analysis(n)
        ref = an.overlaps(a, b)
        torch.cuda.synchronize()
        reserved = torch.cuda.memory_reserved()
        got = analysis_overlaps_noalloc(a, b)
        assert torch.cuda.memory_reserved() == reserved
        np.testing.assert_array_equal(got, ref)
        assert np.all(np.isfinite(got)) and got[1] > 0 and got[5] > 0
        an.close()
    say("case: overlaps without allocation, size checks")
    out = np.zeros(6)
    vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
    for bad_n in (48, 4, 8192):
        rc = lib.tfan_analysis_overlaps_noalloc(bad_n, vp(a.data_ptr()), vp(b.data_ptr()),
                                                out.ctypes.data_as(dp), None)
        assert rc == TFAN_EINVAL, bad_n
        assert b"power of two" in lib.tfan_analysis_noalloc_last_error()
    with pytest.raises(TfanError):
        analysis_overlaps_noalloc(a[:, :16, :16].contiguous(), b[:, :16, :32].contiguous())
