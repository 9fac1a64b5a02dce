"""The seeded 64-member parameter sweep (square grids of 128, 256 and 512 sites,
activity, tumbling parameter, elastic constant and composition drawn uniformly) run
as one batch through the C ABI for 10,000 coupled steps.

Checked: one member of each grid size against the FP64 C oracle at step 100
(relative L2 <= 1e-4 per field, the bar of the plain path); every member's health
flags at step 10,000; and the drift of each member's total composition sum(phi),
which the flux-form central differences conserve exactly, so that only float32
rounding moves it (measured drift and bound stated below)."""
import sys

import numpy as np
import pytest

from oracle.coracle import COracle
from paper_2511_00445_amd.workloads import initial_fields, sweep_members

pytestmark = pytest.mark.gpu
TOL = 1e-4
STEPS = 10000


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_sweep_64_members_10000_steps(gpu):
    from paper_2511_00445_amd import Batch
    members = sweep_members()
    sizes = [m["params"]["nx"] for m in members]
    say(f"case: sweep of {len(members)} members, sizes {sorted(set(sizes))}, {STEPS} steps")
    b = Batch([m["params"] for m in members])
    ics = []
    for i, m in enumerate(members):
        p = m["params"]
        ic = initial_fields(p["nx"], p["ny"], seed=m["seed"], phi_mean=m["phi_mean"])
        ics.append(ic)
        b.init_fields(i, **ic)
    phi0 = [b.diagnostics(i)["phi_sum"] for i in range(len(members))]
    b.step(100)
    # one member of each size against the C oracle
    for n in (128, 256, 512):
        i = sizes.index(n)
        say(f"case: sweep member {i} ({n}x{n}) vs the C oracle at step 100")
        o = COracle(members[i]["params"])
        o.init_fields(**ics[i])
        o.step(100)
        of, g = o.get_fields(), b.get_fields(i)
        for k in ("phi", "qxx", "qxy", "u_a", "u_p"):
            e = float(np.linalg.norm(g[k] - of[k]) / np.linalg.norm(of[k]))
            assert e <= TOL, (i, n, k, e)
    b.step(STEPS - 100)
    b.sync()
    worst = 0.0
    for i, m in enumerate(members):
        d = b.diagnostics(i)
        assert d["status"] == 0, (i, d)
        assert d["step"] == STEPS
        n = m["params"]["nx"] * m["params"]["ny"]
        # The flux-form update conserves sum(phi) exactly in exact arithmetic; in
        # float32 the drift is systematic, not a random walk: inside the bulk
        # phases (|phi| ~ 1, ulp 6e-8) the coarsening flux makes increments below
        # half an ulp, which round away while their sign is set by the mass
        # transport.  Member 15 measured 1.13e-5 per site at 10,000 steps;
        # bound 5e-5 per site.
        drift = abs(d["phi_sum"] - phi0[i]) / n
        worst = max(worst, drift)
        assert drift <= 5e-5, (i, drift)
    say(f"sweep: all {len(members)} members healthy at step {STEPS}; worst phi drift per site {worst:.2e}")
