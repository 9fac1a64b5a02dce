"""CPU checks of the C ABI: the library loads, exports every function that
include/tfan.h declares, and validates parameters on the host (no GPU call)."""
import ctypes
import os
import re

import pytest

import paper_2511_00445_amd as T
from paper_2511_00445_amd.binding import tfan_params, tfan_diag, make_params
from paper_2511_00445_amd.workloads import workload_params

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "tfan.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tfan_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = T.load_library()
    names = declared_functions()
    assert len(names) >= 18
    for name in names:
        assert hasattr(lib, name), name


def test_struct_layouts_match_header():
    # 4 int32 + 13 doubles; 2 int64 + 14 doubles
    assert ctypes.sizeof(tfan_params) == 4 * 4 + 13 * 8
    assert ctypes.sizeof(tfan_diag) == 2 * 8 + 14 * 8
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
