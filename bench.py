"""Throughput of the coupled two-fluid active-nematic step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large_2048]

Prints one JSON line: MLUPS (million lattice-site updates per second, one update
= one coupled step of one site: both lattice-Boltzmann fluids plus all
finite-difference sub-steps), the HBM roofline of the dominant kernel measured
with HIP events on the solver's stream, and the FP64 oracle timed on the host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
ANALYSIS_BYTES_PER_SITE = 52 + 5 * 2 * 16 + 48 + 24 + 8  # one observables snapshot (bench_analysis)
# fp32 vector peak without packed fp32 instructions (the build disables them):
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
VALU_F32_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# Algorithmic bytes per lattice site (float32 storage) as the method defines them:
# the whole coupled step reads and writes 2 fluids x 9 populations and phi, Qxx, Qxy
# (168 B).  The collision kernel's share is the populations (144 B) and the read of
# phi/Q (12 B); the frozen velocities u_a, u_c it writes (16 B) link the collision
# and sub-step kernels of this design and are reported as overhead, not counted.
ALG_BYTES = {
    "step": 168,        # 2*9*4*2 + 3*4*2
    "collide": 156,     # populations read + written (144), phi/Q read (12)
    "substep": 24,      # sub-step launch: phi/Q read and written
    "substeps": 24,     # blocked sub-steps: phi/Q read and written once per launch
}
OVERHEAD_BYTES = {"collide": 16, "substep": 16, "substeps": 16}   # u_a/u_c written, then read
# Arithmetic operations per site of one finite-difference sub-step, as the method
# defines them (no halo recomputation): Cahn-Hilliard 29 (mu 11, div(phi u_c) 9,
# lap mu 5, update 4), Beris-Edwards 81 (W 8, its parts 7, LdG factor 6, lap Q
# and H 16, S(W, Q) 18, advection 16, update 10).
SUBSTEP_FLOPS = 110
BOUND = {"collide": "hbm", "substep": "hbm", "substeps": "alu"}


def shader_clock_mhz():
    """Current shader (GFX) clock of GPU 0 in MHz from amdsmi, or None."""
    try:
        import amdsmi
        amdsmi.amdsmi_init()
        h = amdsmi.amdsmi_get_processor_handles()[0]
        return int(amdsmi.amdsmi_get_clock_info(h, amdsmi.AmdSmiClkType.GFX)["clk"])
    except Exception:
        return None


def source_hash() -> str:
    """Hash of the solver's kernel sources (the counter summary is only valid for them)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2511_00445_amd", "csrc")
    for name in ("tfan_internal.h", "tfan_kernels.hip"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else float(k["bytes_per_launch"])


# Kernels whose HBM traffic profiles/traffic.json records (float32 populations,
# default launch shape), and a pattern of their name in the counter output (a
# defaulted template argument may or may not be printed).
TRAFFIC_KERNELS = {"collide": "k_collide<false, float, 2>", "substeps": "k_fd_pair<40, 5>"}
TRAFFIC_NAMES = {"collide": r"::k_collide<false, float, 2(, false)?>\(", "substeps": r"::k_fd_pair<40, 5>\("}


def write_traffic(root_dir: str, sites: int = 2048 * 2048, out_path: str = ""):
    """profiles/traffic.json from four rocprofv3 --pmc runs under root_dir:
    pmc_step_FETCH / pmc_step_WRITE (this benchmark, FETCH_SIZE / WRITE_SIZE) and
    pmc_copy_FETCH / pmc_copy_WRITE (--calibrate-copy 1024).  Each counter is scaled
    by what it reads for the plain 1 GiB copy."""
    import csv
    import glob
    import re

    def means(sub, counter):
        (path,) = glob.glob(os.path.join(root_dir, sub, "*counter_collection.csv"))
        acc = {}
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                name = r["Kernel_Name"]
                if name.startswith("__amd_rocclr_copyBuffer"):
                    key = "copy"
                else:
                    key = next((k for k, v in TRAFFIC_NAMES.items() if re.search(v, name)), None)
                if key:
                    acc.setdefault(key, []).append(float(r["Counter_Value"]))
        return {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}

    nbytes = 1 << 30
    fetch, write = means("pmc_step_FETCH", "FETCH_SIZE"), means("pmc_step_WRITE", "WRITE_SIZE")
    cf, cw = means("pmc_copy_FETCH", "FETCH_SIZE")["copy"][0], means("pmc_copy_WRITE", "WRITE_SIZE")["copy"][0]
    fs, ws = nbytes / (cf * 1024), nbytes / (cw * 1024)
    rec = {"source_hash": source_hash(),
           "workload": "large_2048 (2048x2048, n_sub=5, default launch shape), bench.py --steps 25 --warmup 5 "
                       "under rocprofv3 --pmc, one counter per run",
           "calibration": {"kernel": "__amd_rocclr_copyBuffer, 1 GiB device copy (bench.py --calibrate-copy 1024)",
                           "FETCH_SIZE_KiB_per_launch": round(cf, 1), "WRITE_SIZE_KiB_per_launch": round(cw, 1),
                           "bytes_read": nbytes, "bytes_written": nbytes,
                           "fetch_scale": round(fs, 4), "write_scale": round(ws, 4)},
           "kernels": {}}
    for key, kname in TRAFFIC_KERNELS.items():
        (fk, nd), (wk, _) = fetch[key], write[key]
        rd, wr = fk * 1024 * fs, wk * 1024 * ws
        rec["kernels"][key] = {"kernel": kname, "dispatches": nd, "FETCH_SIZE_KiB": round(fk, 1),
                               "WRITE_SIZE_KiB": round(wk, 1), "bytes_per_launch": int(round(rd + wr)),
                               "bytes_per_site": round((rd + wr) / sites, 2),
                               "read_bytes_per_site": round(rd / sites, 2), "write_bytes_per_site": round(wr / sites, 2)}
    with open(out_path or os.path.join(ROOT, "profiles", "traffic.json"), "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))
    return rec


def cpu_baseline(params, ic, budget_s: float, single_core_s: float = 0.0):
    """The FP64 C oracle (oracle/coracle.c, OpenMP over rows), unchanged, on the same
    grid: whole coupled steps until the time budget is used, with every host thread;
    with single_core_s > 0, the same again on one thread within that budget."""
    from oracle.coracle import COracle, set_threads, threads

    def timed(budget):
        o = COracle(params)
        o.init_fields(ic["phi"], ic["qxx"], ic["qxy"])
        steps, t0 = 0, time.perf_counter()
        while True:
            o.step(1)
            steps += 1
            el = time.perf_counter() - t0
            if el * (steps + 1) / steps > budget:
                return steps, el

    sites = params["nx"] * params["ny"]
    steps, el = timed(budget_s)
    out = {"value": round(sites * steps / el / 1e6, 3), "unit": "MLUPS", "cores": threads(), "kind": "oracle",
           "sample": f"{steps} coupled steps of the full {params['nx']}x{params['ny']} grid, FP64 C oracle "
                     f"with {threads()} OpenMP threads, {el:.1f} s"}
    if single_core_s > 0:
        n = threads()
        set_threads(1)
        try:
            s1, e1 = timed(single_core_s)
        finally:
            set_threads(n)
        out["single_core"] = {"value": round(sites * s1 / e1 / 1e6, 3), "unit": "MLUPS", "cores": 1,
                              "sample": f"{s1} coupled steps of the same grid on one thread, {e1:.1f} s"}
    return out


def bench_sweep(args):
    """64 independent simulations of sizes 128^2/256^2/512^2 with seeded parameters:
    batched (one launch per phase for all members, autotuned launch shape) against the
    same members stepped one after another as single simulations."""
    import torch
    from paper_2511_00445_amd import Batch, Sim
    from paper_2511_00445_amd.workloads import initial_fields, sweep_members
    members = sweep_members()
    sites = sum(m["params"]["nx"] * m["params"]["ny"] for m in members)
    b = Batch([m["params"] for m in members])
    for i, m in enumerate(members):
        p = m["params"]
        b.init_fields(i, **initial_fields(p["nx"], p["ny"], seed=m["seed"], phi_mean=m["phi_mean"]))
    tuned_ms = b.autotune(steps=5)
    b.step(args.warmup)
    b.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(args.steps)
    b.sync()
    wall = time.perf_counter() - t0
    bad = [i for i in range(len(members)) if b.diagnostics(i)["status"] != 0]
    if bad:
        raise SystemExit(f"unhealthy batch members: {bad}")
    # the same steps in one persistent launch (all members, all steps)
    torch.cuda.synchronize()
    tp = time.perf_counter()
    b.step_persistent(args.steps)
    b.sync()
    wall_p = time.perf_counter() - tp
    persist_blocks = b.persistent_blocks()
    tuning = b.get_tuning()
    b.close()
    sims = []
    for m in members:
        p = m["params"]
        s = Sim(p)
        s.set_tuning(*tuning)
        s.init_fields(**initial_fields(p["nx"], p["ny"], seed=m["seed"], phi_mean=m["phi_mean"]))
        sims.append(s)
    for s in sims:
        s.step(args.warmup)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for s in sims:
        s.step(args.steps)
    torch.cuda.synchronize()
    wall_seq = time.perf_counter() - t1
    out = {"metric": "MLUPS per coupled step (batched sweep)", "value": round(sites * args.steps / wall / 1e6, 1),
           "unit": "MLUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(wall / args.steps * 1e3, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"sweep_64: {len(members)} members, sizes 128/256/512, {sites} sites",
                      "tuning": {"collide_rows": tuning[0], "fd_shape": tuning[1]},
                      "autotune_ms_per_step": round(tuned_ms, 4)},
           "sequential_value": round(sites * args.steps / wall_seq / 1e6, 1),
           "batch_speedup": round(wall_seq / wall, 3),
           "persistent_launch": {"value": round(sites * args.steps / wall_p / 1e6, 1), "unit": "MLUPS",
                                 "ms_per_step": round(wall_p / args.steps * 1e3, 4), "blocks": persist_blocks}}
    print(json.dumps(out), flush=True)


# multiply-adds per site of one surrogate forward pass (7 -> 48 x5 -> 7, 3x3)
CNN_MACS_PER_SITE = 48 * 7 * 9 + 4 * 48 * 48 * 9 + 7 * 48 * 9
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense bf16 matrix peak


def bench_surrogate(args):
    """Surrogate-accelerated coarsening at 1024x1024 (zeta = 0.01, seed 7) against the
    plain path on the same GPU: plain solver to step 6,000, then --deploy-steps
    lattice steps (default 1,005,000, whole calls of k + relax steps) both ways; the
    network is trained first on 256x256 trajectories by the library's own kernels."""
    import numpy as np
    import torch
    from paper_2511_00445_amd import Cnn
    from paper_2511_00445_amd import surrogate as S
    from paper_2511_00445_amd.workloads import base_params, initial_fields
    print("[bench] training the surrogate on 256x256 trajectories", file=sys.stderr, flush=True)
    t1 = args.train_t1 or S.TRAIN_T1
    theta, s_in, s_out, losses, train_s = S.train_surrogate(base_params(256, 256, zeta=0.01), list(S.TRAIN_SEEDS),
                                                            S.TRAIN_T0, t1, steps=args.train_steps, batch=8)
    n = 1024
    p = base_params(n, n, zeta=0.01)
    call = S.K_STEPS + S.RELAX_STEPS
    every = call * 200
    span = every * max(1, -(-args.deploy_steps // every))
    print(f"[bench] plain and surrogate runs at 1024x1024, steps 6000-{6000 + span}", file=sys.stderr, flush=True)
    r = S.deploy_compare(p, 7, theta, s_in, s_out, 6000, 6000 + span, every, relax=S.RELAX_STEPS,
                         log=lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True))
    if r["status"] != 0:
        raise SystemExit("surrogate run became unhealthy")
    # forward-pass throughput with HIP events on the network's stream
    net = Cnn(1, n, n)
    net.set_params(theta)
    net.set_scales(s_in, s_out)
    x = torch.zeros((1, 7, n, n), dtype=torch.float32, device="cuda")
    out = torch.empty_like(x)
    for _ in range(3):
        net.forward(x, out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record(net.stream)
    for _ in range(reps):
        net.forward(x, out)
    e1.record(net.stream)
    net.sync()
    fwd_s = e0.elapsed_time(e1) / reps / 1e3
    flops = 2.0 * CNN_MACS_PER_SITE * n * n
    achieved = flops / fwd_s / 1e12
    # last sampled step up to which every sample's L stays within 5% of the plain run's
    dev = np.abs(np.array(r["L_surrogate"]) / np.array(r["L_plain"]) - 1)
    bad = np.flatnonzero(~(dev <= 0.05))
    within_until = 6000 if bad.size and bad[0] == 0 else r["t"][bad[0] - 1] if bad.size else r["t"][-1]
    out_line = {
        "metric": "simulated lattice steps per second, surrogate-accelerated, domain-length error <= 5%",
        "value": round(r["surrogate_steps_per_s"], 1), "unit": "steps/s", "n_gpus": 1,
        "steps": span, "warmup": 6000, "ms_per_step": round(1e3 / r["surrogate_steps_per_s"], 5),
        "higher_is_better": True, "scaling": "strong", "vs_baseline": None, "dtype": "bf16-mfma/f32",
        "data": "synthetic",
        "config": {"workload": f"surrogate_1024: 1024x1024 periodic, zeta=0.01, seed 7, plain to step 6000, then "
                               f"{span} steps of 50-step network jumps + 25 solver steps, solver check every 10 "
                               f"calls, fallback above 5e-2 relative L2 on (phi, Q); trained on 256x256 steps "
                               f"{S.TRAIN_T0}-{t1}",
                   "nx": n, "ny": n, "k": S.K_STEPS, "relax": S.RELAX_STEPS, "parallelism": "single GPU"},
        "plain_steps_per_s": round(r["plain_steps_per_s"], 1), "speedup": round(r["speedup"], 3),
        "max_L_dev": round(r["max_L_dev"], 4), "L_dev_within_5pct": r["max_L_dev"] <= 0.05,
        "L_within_5pct_through_step": within_until,
        "checks": r["checks"], "fallbacks": r["fallbacks"], "failed_checks": r["failed_checks"],
        "relax_rollbacks": r["relax_rollbacks"], "health_rollbacks": r["health_rollbacks"],
        "deep_rollbacks": r["deep_rollbacks"],
        "max_check_error": r["max_check_error"], "train_seconds": round(train_s, 2),
        "train_loss": [round(float(np.mean(losses[:50])), 4), round(float(np.mean(losses[-200:])), 4)],
        "roofline": {"bound": "mfma", "kernel": "cnn_forward (6 convolutions)", "achieved": round(achieved, 1),
                     "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / BF16_PEAK_TFLOPS, 4),
                     "traffic": None, "alg_flops_per_launch": flops, "avg_launch_us": round(fwd_s * 1e6, 2)},
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on the host", file=sys.stderr, flush=True)
        cb = cpu_baseline(p, initial_fields(n, n, seed=7), args.cpu_budget)
        cb["value"] = round(cb["value"] * 1e6 / (n * n), 3)
        cb["unit"] = "steps/s"
        out_line["cpu_baseline"] = cb
    print(json.dumps(out_line), flush=True)


def bench_cnn(args):
    """The surrogate network alone on synthetic inputs (no solver): forward passes at
    1024x1024 (batch 1) and Adam steps at 256x256 (batch 8), timed with HIP events
    on the network's stream.  Used for the network kernels' counters and traces."""
    import numpy as np
    import torch
    from paper_2511_00445_amd import Cnn
    from paper_2511_00445_amd import surrogate as S
    gen = torch.Generator(device="cuda").manual_seed(0)
    theta = S.init_params(0)
    theta[-(48 * 7 * 9 + 7):] = np.random.default_rng(1).uniform(-0.02, 0.02, 48 * 7 * 9 + 7).astype(np.float32)
    ones = np.ones(7, np.float32)
    n = 1024
    net = Cnn(1, n, n)
    net.set_params(theta)
    net.set_scales(ones, ones)
    x = torch.rand((1, 7, n, n), generator=gen, device="cuda") - 0.5
    out = torch.empty_like(x)
    for _ in range(3):
        net.forward(x, out)
    reps = max(1, args.steps // 100)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(net.stream)
    for _ in range(reps):
        net.forward(x, out)
    e1.record(net.stream)
    net.sync()
    fwd_s = e0.elapsed_time(e1) / reps / 1e3
    tr = Cnn(8, 256, 256, train=True)
    tr.set_params(theta)
    tr.set_scales(ones, ones)
    X = torch.rand((16, 7, 256, 256), generator=gen, device="cuda") - 0.5
    T = X + 0.01 * (torch.rand((16, 7, 256, 256), generator=gen, device="cuda") - 0.5)
    idx = np.arange(8, dtype=np.int32)
    tr.train_step(X, T, idx, 1e-4)
    e0.record(tr.stream)
    for _ in range(reps):
        tr.train_step(X, T, idx, 1e-4, want_loss=False)
    e1.record(tr.stream)
    tr.sync()
    train_s = e0.elapsed_time(e1) / reps / 1e3
    flops = 2.0 * CNN_MACS_PER_SITE * n * n
    achieved = flops / fwd_s / 1e12
    out_line = {"metric": "surrogate network forward passes per second (1024x1024, bf16 MFMA)",
                "value": round(1.0 / fwd_s, 2), "unit": "passes/s", "n_gpus": 1, "steps": reps, "warmup": 3,
                "ms_per_step": round(fwd_s * 1e3, 4), "higher_is_better": True, "scaling": "strong",
                "vs_baseline": None, "dtype": "bf16-mfma/f32", "data": "synthetic",
                "config": {"workload": "cnn_1024: forward 1x7x1024x1024; training step 8x7x256x256",
                           "parallelism": "single GPU"},
                "train_step_ms": round(train_s * 1e3, 4),
                "roofline": {"bound": "mfma", "kernel": "cnn_forward (6 convolutions)", "achieved": round(achieved, 1),
                             "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / BF16_PEAK_TFLOPS, 4),
                             "traffic": None, "alg_flops_per_launch": flops, "avg_launch_us": round(fwd_s * 1e6, 2)}}
    net.close()
    tr.close()
    print(json.dumps(out_line), flush=True)


def bench_analysis(args):
    """On-device observables of one 2048x2048 snapshot (spectra + L, correlations,
    defects in one tfan_analysis_all call) against the FP64 numpy oracle on the host,
    same float32 state."""
    import numpy as np
    import torch
    from paper_2511_00445_amd import Analysis, Sim
    from paper_2511_00445_amd.workloads import WORKLOADS, initial_fields, workload_params
    w = WORKLOADS["large_2048"]
    p = workload_params("large_2048")
    n = p["nx"]
    sim = Sim(p)
    sim.init_fields(**initial_fields(n, n, seed=w["seeds"][0]))
    sim.step(args.warmup)
    x = torch.empty((7, n, n), dtype=torch.float32, device="cuda")
    sim.export_state(x)
    sim.sync()
    an = Analysis(n)

    def snapshot():
        an.all(x)

    snapshot()  # warm-up
    reps = max(1, args.steps // 200)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        snapshot()
    torch.cuda.synchronize()
    per = (time.perf_counter() - t0) / reps
    parts = {}
    for name, fn in (("spectra", lambda: an.spectra(x)), ("correlations", lambda: an.correlations(x)),
                     ("defects", lambda: an.defects(x))):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        parts[name] = round((time.perf_counter() - t1) / reps * 1e3, 3)
    # algorithmic bytes of one snapshot, per site: packing (7 state planes read, 3
    # complex fields written: 52 B), five 2D FFTs at two read+write passes of
    # complex64 each (the least an FFT of an array larger than the chip's caches
    # moves: 160 B), power spectra (24 B read, 24 B written), shell sums (pE, pS
    # and two complex correlation maps read: 24 B), defect count (Qxx, Qxy: 8 B)
    alg = ANALYSIS_BYTES_PER_SITE * n * n
    achieved = alg / per / 1e9
    out = {"metric": "analysed snapshots per second (spectra + L, correlations, defects)",
           "value": round(1.0 / per, 2), "unit": "snapshots/s", "n_gpus": 1, "steps": reps, "warmup": args.warmup,
           "ms_per_step": round(per * 1e3, 3), "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
           "dtype": "f32 (fp64 sums)", "data": "synthetic",
           "config": {"workload": f"analysis_2048: one 2048x2048 snapshot of large_2048 after {args.warmup} steps",
                      "nx": n, "ny": n, "parallelism": "single GPU"},
           "ms_per_call": parts,
           "roofline": {"bound": "hbm", "kernel": "whole snapshot (packing, FFT passes, powers, shell sums, defects)",
                        "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                        "alg_bytes_per_launch": alg, "avg_launch_us": round(per * 1e6, 1)}}
    if not args.no_cpu_baseline:
        from oracle import analysis_oracle as A
        xh = x.cpu().numpy().astype(np.float64)
        t2 = time.perf_counter()
        A.spectra(xh)
        A.correlations(xh)
        A.defects(xh)
        el = time.perf_counter() - t2
        out["cpu_baseline"] = {"value": round(1.0 / el, 4), "unit": "snapshots/s", "cores": 1, "kind": "oracle",
                               "sample": f"one 2048x2048 snapshot through the FP64 numpy oracle, {el:.1f} s"}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="large_2048")
    ap.add_argument("--storage", choices=("f32", "f16"), default="f32",
                    help="population storage (f16: binary16 deviations, float32 arithmetic)")
    ap.add_argument("--cpu-budget", type=float, default=25.0)
    ap.add_argument("--settle-s", type=float, default=2.0,
                    help="seconds of untimed steps right before the timed region (clock settle)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--single-core-budget", type=float, default=8.0,
                    help="seconds of the oracle on one thread (0: skip)")
    ap.add_argument("--train-t1", type=int, default=0,
                    help="surrogate_1024: last trajectory step of the training pairs (0: the standard range)")
    ap.add_argument("--deploy-steps", type=int, default=1000000,
                    help="surrogate_1024: lattice steps of the deployment after the plain start")
    ap.add_argument("--train-steps", type=int, default=12000,
                    help="surrogate_1024: Adam steps of the surrogate's training")
    ap.add_argument("--tuning", default="", metavar="C,F",
                    help="launch shape collide_rows,fd_shape (default: the library's)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration)")
    ap.add_argument("--write-traffic", default="", metavar="DIR",
                    help="only write profiles/traffic.json from the four --pmc runs under DIR (no GPU)")
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(args.write_traffic)
        return
    if args.calibrate_copy:
        import torch
        torch.cuda.set_device(0)
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "device copy", "bytes_read": nbytes, "bytes_written": nbytes,
                          "launches": 3}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path "
              "(a y-slab decomposition is described in the design notes).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2511_00445_amd import Sim
    from paper_2511_00445_amd.workloads import WORKLOADS, initial_fields, workload_params

    torch.cuda.set_device(0)
    if args.workload == "sweep_64":
        return bench_sweep(args)
    if args.workload == "surrogate_1024":
        return bench_surrogate(args)
    if args.workload == "analysis_2048":
        return bench_analysis(args)
    if args.workload == "cnn_1024":
        return bench_cnn(args)
    w = WORKLOADS[args.workload]
    p = workload_params(args.workload)
    p["storage"] = 1 if args.storage == "f16" else 0
    nx, ny = p["nx"], p["ny"]
    ic = initial_fields(nx, ny, seed=w["seeds"][0], phi_mean=w["phi_mean"])
    sim = Sim(p, device="cuda:0")
    if args.tuning:
        sim.set_tuning(*[int(v) for v in args.tuning.split(",")])
    tuning = sim.get_tuning()
    sim.init_fields(**ic)
    print(f"[bench] {args.workload}: {nx}x{ny}, warmup {args.warmup}", file=sys.stderr, flush=True)
    sim.step(args.warmup)
    sim.sync()
    # The shader clock idles at a few hundred MHz and needs about a second of load to
    # reach its steady ~2.4 GHz (a 20-step region timed from idle runs ~15% slow), so
    # the device is kept busy with untimed steps for a fixed wall time right before
    # the timed region; reported as its own field, independent of --warmup.
    settle_steps, t_s = 0, time.perf_counter()
    while time.perf_counter() - t_s < args.settle_s:
        sim.step(20)
        sim.sync()
        settle_steps += 20
    clk_before = shader_clock_mhz()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = sim.stream
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    sim.step(args.steps)
    ev1.record(stream)
    sim.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    region_ms = ev0.elapsed_time(ev1)
    clk_after = shader_clock_mhz()
    # Kernel durations in a second pass of the same length right after the timed one,
    # with HIP events around every launch on the solver's stream (kept out of the
    # timed region, whose throughput they would lower).
    fd = tuning[1]
    if fd in (165, 166):
        block = min(p["n_sub"], 5)
    else:
        block = {162: 2, 163: 3}.get(fd, p["n_sub"] if fd in (16, 32) and p["n_sub"] <= 5 else 1)
    launches_per_step = 1 + -(-p["n_sub"] // block)
    sampled = max(args.steps, 20)
    sim.kernel_timing(sampled * launches_per_step)
    ev2, ev3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev2.record(stream)
    sim.step(sampled)
    ev3.record(stream)
    ktimes = sim.kernel_times()
    sim.kernel_timing(0)
    timed_pass_ms = ev2.elapsed_time(ev3)
    diag = sim.diagnostics()
    if diag["status"] != 0:
        raise SystemExit(f"benchmark state is unhealthy: status {diag['status']}")
    print(f"[bench] timed {args.steps} steps in {wall:.4f} s", file=sys.stderr, flush=True)

    sites = nx * ny
    mlups = sites * args.steps / wall / 1e6
    alg_bytes = dict(ALG_BYTES)
    if p["storage"] == 1:  # populations at 2 bytes
        alg_bytes["step"] -= 72
        alg_bytes["collide"] -= 72
    sub_per_launch = {"substep": 1.0}
    if "substeps" in ktimes and ktimes["substeps"][1] > 0:
        sub_per_launch["substeps"] = p["n_sub"] * sampled / ktimes["substeps"][1]

    def roofline(name):
        ms_tot, count = ktimes[name]
        avg_s = ms_tot / count / 1e3
        if BOUND[name] == "alu":
            flops = SUBSTEP_FLOPS * sub_per_launch[name] * sites
            achieved = flops / avg_s / 1e12
            return {"bound": "alu", "kernel": name, "achieved": round(achieved, 2), "peak": round(VALU_F32_PEAK_TFLOPS, 1),
                    "unit": "TFLOP/s", "frac": round(achieved / VALU_F32_PEAK_TFLOPS, 4),
                    "traffic": measured_traffic(name) if p["storage"] == 0 else None,
                    "alg_flops_per_launch": flops, "avg_launch_us": round(avg_s * 1e6, 2),
                    "hbm_alg_bytes_per_launch": alg_bytes[name] * sites,
                    "overhead_bytes_per_launch": OVERHEAD_BYTES[name] * sites}
        alg = alg_bytes[name] * sites
        achieved = alg / avg_s / 1e9
        return {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(name) if p["storage"] == 0 else None,
                "alg_bytes_per_launch": alg, "avg_launch_us": round(avg_s * 1e6, 2),
                "overhead_bytes_per_launch": OVERHEAD_BYTES[name] * sites}

    # dominant kernel: largest total time in the timed region
    hot = [k for k, v in ktimes.items() if v[1] > 0 and k in BOUND]
    name = max(hot, key=lambda k: ktimes[k][0])
    step_gbs = alg_bytes["step"] * sites * args.steps / wall / 1e9
    out = {
        "metric": "MLUPS per coupled step",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if p["storage"] == 0 else "f16-storage/f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {nx}x{ny} periodic, "
                               f"{'plain float32' if p['storage'] == 0 else 'binary16-storage'} path, "
                               f"zeta={p['zeta']}, n_sub={p['n_sub']}, seed {w['seeds'][0]}",
                   "nx": nx, "ny": ny, "n_sub": p["n_sub"], "parallelism": "single GPU",
                   "tuning": {"collide_rows": tuning[0], "fd_shape": tuning[1]}},
        "roofline": roofline(name),
        "roofline_kernels": {k: roofline(k) for k in hot},
        "step_roofline": {"alg_bytes_per_site": alg_bytes["step"], "achieved": round(step_gbs, 1),
                          "frac": round(step_gbs / HBM_PEAK_GBS, 4)},
        "kernels_ms": {k: [round(v[0], 3), v[1]] for k, v in ktimes.items() if v[1] > 0},
        "kernel_sum_ms_per_step": round(sum(v[0] for k, v in ktimes.items() if k in BOUND) / sampled, 5),
        "event_region_ms": round(region_ms, 3),
        "kernel_timing_pass": {"steps": sampled, "ms_per_step": round(timed_pass_ms / sampled, 5)},
        "clock_settle": {"seconds": args.settle_s, "untimed_steps": settle_steps},
        "gpu_clock_mhz": {"before": clk_before, "after": clk_after},
        "source_hash": source_hash(),
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(p, ic, args.cpu_budget, args.single_core_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
