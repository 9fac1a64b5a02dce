"""Host-side checks of bench.py's contract (no GPU): a request for more than one
GPU ends with a message, and the roofline constants are the ones stated."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_roofline_constants():
    b = _bench()
    assert b.HBM_PEAK_GBS == 8000.0
    # 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz, without packed fp32
    assert abs(b.VALU_F32_PEAK_TFLOPS - 78.6432) < 1e-9
    # populations 2 x 9 x 4 B read and written, phi/Qxx/Qxy read and written
    assert b.ALG_BYTES["step"] == 2 * 9 * 4 * 2 + 3 * 4 * 2
    # the collision's share: populations read and written, phi/Q read; the frozen
    # velocities it writes for the sub-step kernel are overhead of the two-kernel split
    assert b.ALG_BYTES["collide"] == 2 * 9 * 4 * 2 + 3 * 4
    assert b.OVERHEAD_BYTES["collide"] == 4 * 4
    assert b.ALG_BYTES["substeps"] == 3 * 4 * 2
    # observables snapshot: packing 7 x 4 read + 3 x 8 written, five 2D FFTs of two
    # read+write passes over complex64, powers 3 x 8 read + 2 x 4 + 2 x 8 written,
    # shell sums 2 x 4 + 2 x 8 read, defects 2 x 4 read
    assert b.ANALYSIS_BYTES_PER_SITE == (7 * 4 + 3 * 8) + 5 * 2 * 2 * 8 + (3 * 8 + 2 * 4 + 2 * 8) + (2 * 4 + 2 * 8) + 2 * 4


def test_traffic_record_matches_sources_or_is_ignored():
    b = _bench()
    t = b.measured_traffic("collide")
    assert t is None or t > 0


def test_traffic_summary_from_counter_files(tmp_path):
    """bench.py --write-traffic: per-launch HBM bytes = FETCH_SIZE and WRITE_SIZE (KiB)
    scaled by what each counter reads for the 1 GiB copy, averaged over dispatches;
    kernel names match with or without the defaulted template argument."""
    import csv
    import bench

    def put(sub, counter, rows):
        d = tmp_path / sub
        d.mkdir()
        with open(d / "x_counter_collection.csv", "w", newline="") as f:
            w = csv.writer(f)
            w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
            for i, (name, v) in enumerate(rows):
                w.writerow([i, name, counter, v])

    col = "void tfan::(anonymous namespace)::k_collide<false, float, 2, false>(tfan::DevParams, ...)"
    col_true = "void tfan::(anonymous namespace)::k_collide<true, float, 2, false>(tfan::DevParams, ...)"
    fd = "void tfan::(anonymous namespace)::k_fd_pair<40, 5>(tfan::DevParams, ...)"
    put("pmc_step_FETCH", "FETCH_SIZE", [(col, 100.0), (col, 120.0), (col_true, 999.0), (fd, 10.0)])
    put("pmc_step_WRITE", "WRITE_SIZE", [(col, 200.0), (col, 200.0), (fd, 20.0)])
    put("pmc_copy_FETCH", "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 524288.0)] * 3)
    put("pmc_copy_WRITE", "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 1048576.0)] * 3)
    rec = bench.write_traffic(str(tmp_path), sites=1024, out_path=str(tmp_path / "t.json"))
    assert rec["calibration"]["fetch_scale"] == 2.0 and rec["calibration"]["write_scale"] == 1.0
    c = rec["kernels"]["collide"]
    assert c["dispatches"] == 2
    assert c["bytes_per_launch"] == (110.0 * 2.0 + 200.0) * 1024
    assert c["bytes_per_site"] == round((110.0 * 2.0 + 200.0), 2)
    assert rec["kernels"]["substeps"]["bytes_per_launch"] == (10.0 * 2.0 + 20.0) * 1024
    assert rec["source_hash"] == bench.source_hash()
