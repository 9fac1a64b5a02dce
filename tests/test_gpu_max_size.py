"""The largest grid the C ABI accepts (nx * ny = 2^28 sites, nx = 32768): every
kernel of a step, the state export and the diagnostics at the index ranges
nothing smaller reaches (row offsets up to 2^28, plane offsets up to 5 * 2^28,
buffer byte offsets up to 2^30), in the benchmark's launch configuration.

The state is exported on the device and only windows are copied to the host;
they are compared with the FP64 oracle run on periodic windows (exact after the
steps taken, a step depending on at most 12 sites per direction), at the corners
and seams where the largest indices occur: float32 to the 1e-4 relative L2 bar,
binary16 population storage to its stated bounds (phi 5e-5, Q 1e-3, u_a 5e-3,
u_p 2.5e-2).
"""
import sys

import numpy as np
import pytest

from tests.windows import window_oracle
from paper_2511_00445_amd.workloads import base_params, initial_fields

pytestmark = pytest.mark.gpu
NX, NY, STEPS, HALF = 32768, 8192, 2, 8
BOUNDS = {0: dict(phi=1e-4, qxx=1e-4, qxy=1e-4, u_a=1e-4, u_p=1e-4),
          1: dict(phi=5e-5, qxx=1e-3, qxy=1e-3, u_a=5e-3, u_p=2.5e-2)}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(g, o):
    return float(np.linalg.norm(g - o) / max(np.linalg.norm(o), 1e-8 * np.sqrt(o.size)))


@pytest.mark.parametrize("storage", [0, 1], ids=["f32", "f16"])
def test_largest_grid_windows_match_oracle(gpu, storage):
    import torch
    from paper_2511_00445_amd import Sim
    say(f"case: max size {NX}x{NY}, {STEPS} steps, storage {storage}")
    p = dict(base_params(NX, NY, zeta=0.02), storage=storage)
    ic = initial_fields(NX, NY, seed=11, phi_noise=0.3, S0=0.3)
    sim = Sim(p)
    sim.init_fields(**ic)
    sim.step(STEPS)
    d = sim.diagnostics()
    assert d["status"] == 0
    assert abs(d["phi_sum"] - float(ic["phi"].sum())) < 1e-4 * float(np.abs(ic["phi"]).sum())
    state = torch.empty((7, NY, NX), dtype=torch.float32, device="cuda")
    sim.export_state(state)
    torch.cuda.synchronize()
    for cx, cy in [(0, 0), (NX - 1, NY - 1), (NX - 5, 3), (7, NY - 2), (NX // 2 + 3, NY // 3)]:
        of, xs, ys = window_oracle(p, ic, cx, cy, HALF, STEPS)
        yi = torch.as_tensor(ys, device="cuda")
        xi = torch.as_tensor(xs, device="cuda")
        w = state.index_select(1, yi).index_select(2, xi).cpu().numpy().astype(np.float64)
        got = {"phi": w[0], "qxx": w[1], "qxy": w[2], "u_a": w[3:5], "u_p": w[5:7]}
        errs = {k: rel_l2(got[k], of[k]) for k in got}
        say(f"  window ({cx},{cy}): {errs}")
        assert all(v <= BOUNDS[storage][k] for k, v in errs.items()), (cx, cy, errs)
    del state
    sim.close()
