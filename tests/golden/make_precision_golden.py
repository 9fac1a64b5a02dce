"""Write tests/golden/stats_large_2048.json: statistics of the FP64 C oracle on the
2048x2048 precision-study grid (seed 4), for zeta in {0.02, 0.005, 0}, every 500
steps up to 3,000: the domain length L, the mixture kinetic energy <|u_c|^2>/2,
octave-band sums of E(k) of u_c up to N/4, and the phi mass sum(phi) / N^2.

Calls only oracle/ (and the seeded input generator).
Usage: python tests/golden/make_precision_golden.py [zeta ...]
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

N, T, EVERY, SEED = 2048, 3000, 500, 4
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "stats_large_2048.json")


def octave_bands(E, kmax):
    out, lo = [], 1
    while 2 * lo <= kmax:
        out.append(float(np.sum(E[lo:2 * lo])))
        lo *= 2
    return out


def run(zeta):
    o = COracle(workload_params("large_2048", zeta=zeta))
    o.init_fields(**initial_fields(N, N, seed=SEED))
    rec = {"t": [], "L": [], "ke_c": [], "bands": [], "phi_mean": []}
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
        rec["phi_mean"].append(float(f["phi"].mean()))
        print(f"zeta {zeta} step {o.step_count} L {rec['L'][-1]:.3f} ke {rec['ke_c'][-1]:.3e} "
              f"({time.time() - t0:.0f} s)", flush=True)
    return rec


if __name__ == "__main__":
    zetas = [float(z) for z in sys.argv[1:]] or [0.02, 0.005, 0.0]
    data = {"workload": "large_2048", "oracle": "oracle/coracle.c (FP64)", "seed": SEED, "steps": T,
            "every": EVERY, "band_edges": [2 ** j for j in range(10)], "zeta": {}}
    if os.path.exists(OUT):
        data = json.load(open(OUT))
    for z in zetas:
        data["zeta"][repr(z)] = run(z)
        data["threads"] = threads()
        json.dump(data, open(OUT, "w"))
