"""CPU checks of the C ABI: the library loads, exports every function that
include/*.h declares, and validates parameters on the host (no GPU call)."""
import ctypes
import os
import re

import pytest

import paper_2511_00445_amd as T
from paper_2511_00445_amd.binding import tfan_params, tfan_diag, make_params
from paper_2511_00445_amd.workloads import workload_params

INCLUDE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
HEADER = os.path.join(INCLUDE, "tfan.h")


def declared_functions(path=HEADER):
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tfan_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = T.load_library()
    headers = sorted(f for f in os.listdir(INCLUDE) if f.endswith(".h"))
    assert "tfan.h" in headers and "tfan_cnn.h" in headers
    names = [n for h in headers for n in declared_functions(os.path.join(INCLUDE, h))]
    assert len(names) >= 30
    for name in names:
        assert hasattr(lib, name), name


def test_struct_layouts_match_header():
    # 4 int32 + 13 doubles; 2 int64 + 15 doubles
    assert ctypes.sizeof(tfan_params) == 4 * 4 + 13 * 8
    assert ctypes.sizeof(tfan_diag) == 2 * 8 + 15 * 8
    text = open(HEADER).read()
    body = re.search(r"typedef struct tfan_params \{(.*?)\} tfan_params;", text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"\b([A-Za-z_][A-Za-z_0-9]*)\s*[,;]", body)
    assert fields == [f for f, _ in tfan_params._fields_]


def test_host_validation():
    p = workload_params("small_64")
    T.check_params(p)
    assert T.workspace_bytes(p) > 64 * 64 * 4 * 40
    for bad in (dict(nx=7), dict(ny=40000), dict(tau_a=0.5), dict(tau_p=0.2), dict(n_sub=0),
                dict(M=-1.0), dict(zeta=float("nan")), dict(rho0=0.0), dict(storage=3)):
        q = dict(p, **bad)
        with pytest.raises(T.TfanError) as e:
            T.check_params(q)
        assert e.value.code == T.TFAN_EINVAL
        assert T.workspace_bytes(q) == 0


def test_create_rejects_without_touching_the_gpu():
    lib = T.load_library()
    p = make_params(workload_params("small_64"))
    h = ctypes.c_void_p()
    assert lib.tfan_create(ctypes.byref(p), None, 10, None, ctypes.byref(h)) == T.TFAN_EINVAL
    assert lib.tfan_create(ctypes.byref(p), ctypes.c_void_p(256), 10, None, ctypes.byref(h)) == T.TFAN_ENOMEM
    assert b"workspace too small" in lib.tfan_last_error(None)
    assert lib.tfan_create(ctypes.byref(p), ctypes.c_void_p(100), 1 << 30, None, ctypes.byref(h)) == T.TFAN_EINVAL
    assert lib.tfan_step(None, 1) == T.TFAN_EINVAL
    assert lib.tfan_kernel_count() >= 2


def test_cnn_host_validation():
    lib = T.load_library()
    assert T.Cnn.param_count() == 89239
    assert lib.tfan_cnn_workspace_bytes(1, 64, 64, 0) > 0
    assert lib.tfan_cnn_workspace_bytes(2, 64, 64, 1) > lib.tfan_cnn_workspace_bytes(2, 64, 64, 0)
    for bad in ((0, 64, 64), (1, 63, 64), (1, 64, 8), (1, 0, 64)):
        assert lib.tfan_cnn_workspace_bytes(*bad, 1) == 0
    h = ctypes.c_void_p()
    assert lib.tfan_cnn_create(1, 64, 64, 0, None, 0, None, ctypes.byref(h)) == T.TFAN_EINVAL
    assert lib.tfan_cnn_create(1, 64, 64, 0, ctypes.c_void_p(256), 10, None, ctypes.byref(h)) == T.TFAN_ENOMEM
    assert b"workspace too small" in lib.tfan_cnn_last_error(None)
