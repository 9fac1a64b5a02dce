"""Long-time statistics on the 512x512 active workload (zeta = 0.01, 20,000 steps):
the GPU path against the FP64 oracle, same seeds.

The flow is chaotic, so pointwise parity is only asked for up to step 100; here
statistics are compared: the domain length L(t), the mixture kinetic energy and
octave-band sums of E(k) up to N/4.  The oracle's seed-to-seed spread (seeds 1-3)
is printed beside every deviation as the noise floor of the statistic.

Windows.  From about step 12,000 a grid-scale (checkerboard) velocity mode, which
the collocated central differences of the scheme leave undamped in the mixture,
grows in both implementations; by the last quarter (15,000-20,000) it carries
a large share of the kinetic energy, its growth phase depends on rounding, and
the oracle's own seed spread is 20-60% in KE and in the low bands.  Hence:
  - L(t) at log-spaced times up to 16,000: within 5% (both storages);
  - steps 9,000-12,000 (the last quarter of the run before the mode holds 1e-3 of
    the velocity variance): mean L, mean KE and every band within 5% (both);
  - last quarter: mean L within 5% (both); float32 also KE and the bands n >= 2
    within 5%; the single-shell band n = 1 and the binary16 KE and bands are
    reported with the seed spread.
"""
import sys

import numpy as np
import pytest

from tests.longstats import at_times, gpu_record, load_golden, rel_dev, window_stats

pytestmark = pytest.mark.gpu
TOL = 0.05
LOG_TIMES = (500, 1000, 2000, 4000, 8000, 16000)
WINDOWS = {"last_quarter": (15000, 20000), "pre_onset": (9000, 12000)}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def seed_spread(golden, t0, t1):
    """Largest relative deviation of one seed's window statistics from the seed mean."""
    ws = [window_stats(r, t0, t1) for r in golden["seeds"].values()]
    out = {}
    for key in ("L", "ke_c"):
        v = np.array([w[key] for w in ws])
        out[key] = float(np.max(np.abs(v - v.mean()) / v.mean()))
    b = np.array([w["bands"] for w in ws])
    out["bands"] = np.max(np.abs(b - b.mean(0)) / b.mean(0), axis=0)
    return out


@pytest.mark.parametrize("storage", [0, 1], ids=["f32", "f16"])
@pytest.mark.parametrize("seed", ["1", "2", "3"])
def test_long_time_statistics(gpu, seed, storage):
    golden = load_golden()
    if seed not in golden["seeds"]:
        pytest.skip(f"no oracle record for seed {seed}")
    ref = golden["seeds"][seed]
    say(f"case: active_512 seed {seed} storage {storage}, {golden['steps']} steps")
    rec = gpu_record(int(seed), storage=storage, steps=golden["steps"], every=golden["every"])
    assert all(s == 0 for s in rec["status"]), rec["status"]
    assert rec["t"] == ref["t"]

    dL = rel_dev(at_times(rec, LOG_TIMES), at_times(ref, LOG_TIMES))
    say(f"L(t) at {LOG_TIMES}: gpu {np.round(at_times(rec, LOG_TIMES), 3).tolist()} "
        f"oracle {np.round(at_times(ref, LOG_TIMES), 3).tolist()} rel dev {np.round(dL, 4).tolist()}")
    assert np.all(dL <= TOL), dL

    for name, (t0, t1) in WINDOWS.items():
        g, o = window_stats(rec, t0, t1), window_stats(ref, t0, t1)
        spread = seed_spread(golden, t0, t1)
        dl = float(rel_dev(g["L"], o["L"]))
        dk = float(rel_dev(g["ke_c"], o["ke_c"]))
        db = rel_dev(g["bands"], o["bands"])
        say(f"{name} [{t0},{t1}]: L dev {dl:.4f} (seed spread {spread['L']:.4f}); "
            f"KE dev {dk:.4f} (spread {spread['ke_c']:.4f}); band devs "
            f"{np.round(db, 4).tolist()} (spread {np.round(spread['bands'], 4).tolist()})")
        assert dl <= TOL, (name, dl)
        if name == "pre_onset":
            assert dk <= TOL and np.all(db <= TOL), (name, dk, db)
        elif storage == 0:
            assert dk <= TOL and np.all(db[1:] <= TOL), (name, dk, db)

    # the grid-scale mode: negligible before the pre-onset window ends in both, and
    # where the oracle's share exceeds 10% the GPU run shows it too
    t = np.asarray(ref["t"])
    pre = t <= WINDOWS["pre_onset"][1]
    assert max(np.asarray(ref["nyq"])[pre]) < 1e-3 and max(np.asarray(rec["nyq"])[pre]) < 1e-3
    late = np.asarray(ref["nyq"]) > 0.1
    if late.any():
        assert np.all(np.asarray(rec["nyq"])[late] > 0.02), (np.asarray(rec["nyq"])[late])
