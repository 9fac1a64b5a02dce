"""Write tests/golden/stats_active_512.json: long-time statistics of the FP64 C oracle
on the 512x512 active workload (zeta = 0.01), seeds 1-3.

Calls only oracle/ (and the seeded input generator).  For each seed, every 500 steps
up to 20,000:
  L      domain length of phi (Results, coarsening length)
  ke_c   mixture kinetic energy <|u_c|^2>/2
  bands  octave-band sums of the shell spectrum E(n) of u_c, bands [1,2), [2,4), ...,
         [64,128) (up to N/4)
  nyq    fraction of the variance of u_a,x in the grid-scale rows and columns
         |n_x| >= N/2 - 2 or |n_y| >= N/2 - 2 (tracks a checkerboard velocity mode that
         the collocated central-difference scheme lets grow at late times)
Usage: python tests/golden/make_stats_golden.py [seeds...]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.coracle import COracle, threads  # noqa: E402
from oracle.tfan_oracle import domain_length, energy_spectrum  # noqa: E402
from paper_2511_00445_amd.workloads import initial_fields, workload_params  # noqa: E402

N, T, EVERY = 512, 20000, 500
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "stats_active_512.json")


def octave_bands(E, kmax):
    out, lo = [], 1
    while 2 * lo <= kmax:
        out.append(float(np.sum(E[lo:2 * lo])))
        lo *= 2
    return out


def grid_scale_fraction(g):
    F = np.abs(np.fft.fft2(g - g.mean())) ** 2
    n = g.shape[0]
    f = np.abs(np.fft.fftfreq(n) * n)
    m = (f[None, :] >= n // 2 - 2) | (f[:, None] >= n // 2 - 2)
    return float(F[m].sum() / max(F.sum(), 1e-300))


def run(seed):
    p = workload_params("active_512")
    o = COracle(p)
    o.init_fields(**initial_fields(N, N, seed=seed))
    rec = {"t": [], "L": [], "ke_c": [], "bands": [], "nyq": []}
    t0 = time.time()
    while o.step_count < T:
        o.step(EVERY)
        f = o.get_fields()
        c1 = 0.5 * (1 + f["phi"])
        uc = c1 * f["u_a"] + (1 - c1) * f["u_p"]
        rec["t"].append(o.step_count)
        rec["L"].append(domain_length(f["phi"]))
        rec["ke_c"].append(float(0.5 * (uc ** 2).sum(0).mean()))
        rec["bands"].append(octave_bands(energy_spectrum(uc), N // 4))
        rec["nyq"].append(grid_scale_fraction(f["u_a"][0]))
        print(f"seed {seed} step {o.step_count} L {rec['L'][-1]:.3f} ke {rec['ke_c'][-1]:.3e} "
              f"nyq {rec['nyq'][-1]:.2e} ({time.time() - t0:.0f} s)", flush=True)
    return rec


if __name__ == "__main__":
    seeds = [int(s) for s in sys.argv[1:]] or [1, 2, 3]
    data = {"workload": "active_512", "oracle": "oracle/coracle.c (FP64)", "steps": T,
            "every": EVERY, "band_edges": [2 ** j for j in range(8)], "seeds": {}}
    if os.path.exists(OUT):
        old = json.load(open(OUT))
        if old.get("band_edges") == data["band_edges"]:
            data = old
    for s in seeds:
        data["seeds"][str(s)] = run(s)
        data["threads"] = threads()
        json.dump(data, open(OUT, "w"))
