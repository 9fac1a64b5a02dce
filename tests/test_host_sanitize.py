"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/hostsan_main.cpp drives every host-side validation path of the C ABI
(parameter checks, workspace sizes, handle set-up, argument checks, the host
array scans of init_fields) without touching a GPU.  The host sources are
compiled with the sanitizers on the host side only (the device code is built
as usual and its kernels are never launched here)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2511_00445_amd", "csrc")
BUILT = os.path.join(ROOT, "paper_2511_00445_amd", "_build")


def _hipcc():
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return path if os.path.exists(path) else None


@pytest.mark.slow
def test_host_code_under_sanitizers(tmp_path):
    cc = _hipcc()
    if cc is None:
        pytest.skip("hipcc not available")
    from paper_2511_00445_amd.build import HIP_FLAGS
    base = [f for f in HIP_FLAGS if f not in ("-O3",)]
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    objs = []
    for src in ("tfan.cpp", "cnn.cpp", "analysis.cpp", "overlaps_noalloc.hip"):
        obj = str(tmp_path / (src + ".o"))
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        subprocess.run([cc, "-O1", "-g"] + base + san + lang + ["-c", os.path.join(CSRC, src), "-o", obj],
                       check=True, capture_output=True)
        objs.append(obj)
    for src in ("tfan_kernels.hip", "cnn_kernels.hip", "analysis_kernels.hip"):
        obj = os.path.join(BUILT, src.replace(".hip", ".o"))
        if not os.path.exists(obj):
            obj = str(tmp_path / (src + ".o"))
            subprocess.run([cc] + HIP_FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj],
                           check=True, capture_output=True)
        objs.append(obj)
    main = str(tmp_path / "main.o")
    subprocess.run([cc, "-O1", "-g", "-std=c++17"] + san + ["-I", os.path.join(ROOT, "include"), "-c",
                    os.path.join(ROOT, "tests", "hostsan_main.cpp"), "-o", main], check=True, capture_output=True)
    exe = str(tmp_path / "hostsan")
    subprocess.run([cc, "--offload-arch=gfx950"] + san + ["-o", exe, main] + objs, check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report[-4000:]
    assert "host checks passed" in r.stdout
    assert "ERROR: AddressSanitizer" not in report and "runtime error" not in report, report[-4000:]
