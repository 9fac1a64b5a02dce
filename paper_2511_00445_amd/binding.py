"""Thin ctypes binding of libtfan.so (include/tfan.h).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch supplies the device workspace and the stream.  There is no CPU
fallback: without the built library or a GPU the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtfan.so")

TFAN_OK, TFAN_EINVAL, TFAN_ENOMEM, TFAN_EHIP, TFAN_ENONFINITE, TFAN_EUNSTABLE = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "TFAN_OK", -1: "TFAN_EINVAL", -2: "TFAN_ENOMEM", -3: "TFAN_EHIP",
                -4: "TFAN_ENONFINITE", -5: "TFAN_EUNSTABLE"}
TFAN_STORAGE_F32, TFAN_STORAGE_F16 = 0, 1


class tfan_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("n_sub", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("rho0", ctypes.c_double), ("tau_a", ctypes.c_double),
                ("tau_p", ctypes.c_double), ("gamma", ctypes.c_double), ("A_ch", ctypes.c_double),
                ("kappa", ctypes.c_double), ("M", ctypes.c_double), ("A0", ctypes.c_double),
                ("gamma_ldg", ctypes.c_double), ("K", ctypes.c_double), ("lam", ctypes.c_double),
                ("Gamma", ctypes.c_double), ("zeta", ctypes.c_double)]


class tfan_diag(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("nonfinite", ctypes.c_int64)] + [
        (k, ctypes.c_double) for k in ("phi_sum", "phi_sq_sum", "mass_a", "mass_p", "ke_a", "ke_p",
                                       "ke_c", "ua_sq", "uc_sq", "enstrophy_a", "enstrophy_c",
                                       "elastic", "s_mean", "umax", "phi_absmax")]


class TfanError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None
_P = ctypes.POINTER
_vp = ctypes.c_void_p
_dp = _P(ctypes.c_double)


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libtfan.so once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2511_00445_amd.build`")
    # torch ships its own HIP runtime under the same soname; loading torch first
    # makes libtfan.so bind to that one copy instead of a second runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    sigs = {
        "tfan_check_params": (ctypes.c_int, [_P(tfan_params)]),
        "tfan_workspace_bytes": (ctypes.c_size_t, [_P(tfan_params)]),
        "tfan_create": (ctypes.c_int, [_P(tfan_params), _vp, ctypes.c_size_t, _vp, _P(_vp)]),
        "tfan_init_fields": (ctypes.c_int, [_vp, _dp, _dp, _dp, _dp, _dp]),
        "tfan_step": (ctypes.c_int, [_vp, ctypes.c_int64]),
        "tfan_get_fields": (ctypes.c_int, [_vp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]),
        "tfan_diagnostics": (ctypes.c_int, [_vp, _P(tfan_diag)]),
        "tfan_state_bytes": (ctypes.c_size_t, [_vp]),
        "tfan_get_state": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
        "tfan_set_state": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
        "tfan_sync": (ctypes.c_int, [_vp]),
        "tfan_step_count": (ctypes.c_int64, [_vp]),
        "tfan_kernel_timing": (ctypes.c_int, [_vp, ctypes.c_int64]),
        "tfan_kernel_times": (ctypes.c_int, [_vp, _dp, _P(ctypes.c_int64), ctypes.c_int]),
        "tfan_kernel_count": (ctypes.c_int, []),
        "tfan_set_tuning": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32]),
        "tfan_get_tuning": (ctypes.c_int, [_vp, _P(ctypes.c_int32), _P(ctypes.c_int32)]),
        "tfan_autotune": (ctypes.c_int, [_vp, ctypes.c_int32, _dp]),
        "tfan_batch_workspace_bytes": (ctypes.c_size_t, [_P(tfan_params), ctypes.c_int32]),
        "tfan_batch_create": (ctypes.c_int, [_P(tfan_params), ctypes.c_int32, _vp, ctypes.c_size_t, _vp, _P(_vp)]),
        "tfan_batch_count": (ctypes.c_int, [_vp]),
        "tfan_batch_init_fields": (ctypes.c_int, [_vp, ctypes.c_int32, _dp, _dp, _dp, _dp, _dp]),
        "tfan_batch_step": (ctypes.c_int, [_vp, ctypes.c_int64]),
        "tfan_batch_step_persistent": (ctypes.c_int, [_vp, ctypes.c_int64]),
        "tfan_batch_persistent_blocks": (ctypes.c_int, [_vp]),
        "tfan_batch_get_fields": (ctypes.c_int, [_vp, ctypes.c_int32, _dp, _dp, _dp, _dp, _dp, _dp, _dp]),
        "tfan_batch_diagnostics": (ctypes.c_int, [_vp, ctypes.c_int32, _P(tfan_diag)]),
        "tfan_batch_set_tuning": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32]),
        "tfan_batch_get_tuning": (ctypes.c_int, [_vp, _P(ctypes.c_int32), _P(ctypes.c_int32)]),
        "tfan_batch_autotune": (ctypes.c_int, [_vp, ctypes.c_int32, _dp]),
        "tfan_batch_sync": (ctypes.c_int, [_vp]),
        "tfan_batch_destroy": (None, [_vp]),
        "tfan_batch_last_error": (ctypes.c_char_p, [_vp]),
        "tfan_kernel_name": (ctypes.c_char_p, [ctypes.c_int]),
        "tfan_exchange_bytes": (ctypes.c_size_t, [_vp, ctypes.c_int32]),
        "tfan_export_state": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, ctypes.c_int32]),
        "tfan_import_state": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64]),
        "tfan_cnn_param_count": (ctypes.c_int64, []),
        "tfan_cnn_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                       ctypes.c_int32]),
        "tfan_cnn_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp,
                                           ctypes.c_size_t, _vp, _P(_vp)]),
        "tfan_cnn_set_params": (ctypes.c_int, [_vp, _P(ctypes.c_float)]),
        "tfan_cnn_get_params": (ctypes.c_int, [_vp, _P(ctypes.c_float)]),
        "tfan_cnn_set_scales": (ctypes.c_int, [_vp, _P(ctypes.c_float), _P(ctypes.c_float)]),
        "tfan_cnn_forward": (ctypes.c_int, [_vp, _vp, _vp]),
        "tfan_cnn_gradients": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int64, _P(ctypes.c_int32),
                                              _P(ctypes.c_float), _dp]),
        "tfan_cnn_train_step": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int64, _P(ctypes.c_int32), ctypes.c_float,
                                               _dp]),
        "tfan_cnn_compare": (ctypes.c_int, [_vp, _vp, _vp, _dp]),
        "tfan_cnn_sync": (ctypes.c_int, [_vp]),
        "tfan_cnn_destroy": (None, [_vp]),
        "tfan_cnn_last_error": (ctypes.c_char_p, [_vp]),
        "tfan_analysis_shells": (ctypes.c_int32, [ctypes.c_int32]),
        "tfan_analysis_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32]),
        "tfan_analysis_create": (ctypes.c_int, [ctypes.c_int32, _vp, ctypes.c_size_t, _vp, _P(_vp)]),
        "tfan_analysis_spectra": (ctypes.c_int, [_vp, _vp, _dp, _dp, _dp, _dp, _dp]),
        "tfan_analysis_correlations": (ctypes.c_int, [_vp, _vp, _dp, _dp, _dp, _dp]),
        "tfan_analysis_overlaps": (ctypes.c_int, [_vp, _vp, _vp, _dp]),
        "tfan_analysis_defects": (ctypes.c_int, [_vp, _vp, _P(ctypes.c_int64), _P(ctypes.c_int64)]),
        "tfan_analysis_overlaps_noalloc": (ctypes.c_int, [ctypes.c_int32, _vp, _vp, _dp, _vp]),
        "tfan_analysis_noalloc_last_error": (ctypes.c_char_p, []),
        "tfan_analysis_sync": (ctypes.c_int, [_vp]),
        "tfan_analysis_destroy": (None, [_vp]),
        "tfan_analysis_last_error": (ctypes.c_char_p, [_vp]),
        "tfan_destroy": (None, [_vp]),
        "tfan_last_error": (ctypes.c_char_p, [_vp]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def make_params(p: dict) -> tfan_params:
    out = tfan_params()
    for name, typ in tfan_params._fields_:
        if name == "storage":
            out.storage = int(p.get("storage", TFAN_STORAGE_F32))
        else:
            setattr(out, name, int(p[name]) if typ is ctypes.c_int32 else float(p[name]))
    return out


def check_params(p: dict) -> None:
    """Host-only validation (no GPU call); raises TfanError."""
    lib = load_library()
    rc = lib.tfan_check_params(ctypes.byref(make_params(p)))
    if rc != TFAN_OK:
        raise TfanError(rc, lib.tfan_last_error(None).decode())


def workspace_bytes(p: dict) -> int:
    return int(load_library().tfan_workspace_bytes(ctypes.byref(make_params(p))))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _check_dev(t, shape=None):
    """A contiguous float32 tensor on a HIP device (optionally of a given trailing shape)."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise TfanError(TFAN_EINVAL, "expected a contiguous float32 device tensor")
    if shape is not None and tuple(t.shape[-len(shape):]) != tuple(shape):
        raise TfanError(TFAN_EINVAL, f"expected trailing shape {shape}, got {tuple(t.shape)}")


def _exchange_planes(t, ny, nx) -> int:
    """Plane count (7 or 9) of a state exchange tensor [planes][ny][nx]."""
    _check_dev(t)
    if t.dim() != 3 or tuple(t.shape[1:]) != (ny, nx) or t.shape[0] not in (7, 9):
        raise TfanError(TFAN_EINVAL, f"expected a [7 or 9][{ny}][{nx}] tensor, got {tuple(t.shape)}")
    return int(t.shape[0])


def _f64(a, shape):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != shape:
        a = a.reshape(shape)
    return a


class Sim:
    """One solver on one device and stream; the device workspace is a torch tensor."""

    def __init__(self, params: dict, device=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the solver runs only on the GPU")
        self.lib = load_library()
        self.params = dict(params)
        self.nx, self.ny = int(params["nx"]), int(params["ny"])
        cp = make_params(params)
        rc = self.lib.tfan_check_params(ctypes.byref(cp))
        if rc != TFAN_OK:
            raise TfanError(rc, self.lib.tfan_last_error(None).decode())
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        nbytes = int(self.lib.tfan_workspace_bytes(ctypes.byref(cp)))
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._handle = _vp()
        with torch.cuda.device(self.device):
            rc = self.lib.tfan_create(ctypes.byref(cp), _vp(aligned), nbytes, _vp(self.stream.cuda_stream),
                                      ctypes.byref(self._handle))
        if rc != TFAN_OK:
            raise TfanError(rc, self.lib.tfan_last_error(None).decode())

    # -- helpers -----------------------------------------------------------------
    def _check(self, rc):
        if rc != TFAN_OK:
            raise TfanError(rc, self.lib.tfan_last_error(self._handle).decode())

    @property
    def handle(self):
        return self._handle

    # -- the ABI -------------------------------------------------------------------
    def init_fields(self, phi, qxx, qxy, u_a=None, u_p=None):
        s = (self.ny, self.nx)
        arrs = [_f64(phi, s), _f64(qxx, s), _f64(qxy, s), _f64(u_a, (2,) + s), _f64(u_p, (2,) + s)]
        self._check(self.lib.tfan_init_fields(self._handle, *[_ptr(a) for a in arrs]))

    def step(self, n: int = 1):
        self._check(self.lib.tfan_step(self._handle, int(n)))

    def get_fields(self) -> dict:
        s = (self.ny, self.nx)
        out = dict(phi=np.empty(s), qxx=np.empty(s), qxy=np.empty(s), u_a=np.empty((2,) + s),
                   u_p=np.empty((2,) + s), rho_a=np.empty(s), rho_p=np.empty(s))
        self._check(self.lib.tfan_get_fields(self._handle, *[_ptr(out[k]) for k in
                                                             ("phi", "qxx", "qxy", "u_a", "u_p", "rho_a", "rho_p")]))
        return out

    def diagnostics(self) -> dict:
        """Diagnostics sums; 'status' is TFAN_OK, TFAN_ENONFINITE or TFAN_EUNSTABLE."""
        d = tfan_diag()
        rc = self.lib.tfan_diagnostics(self._handle, ctypes.byref(d))
        if rc not in (TFAN_OK, TFAN_ENONFINITE, TFAN_EUNSTABLE):
            self._check(rc)
        out = {name: getattr(d, name) for name, _ in tfan_diag._fields_}
        out["status"] = rc
        return out

    def state_bytes(self) -> int:
        return int(self.lib.tfan_state_bytes(self._handle))

    def get_state(self) -> np.ndarray:
        buf = np.empty(self.state_bytes(), dtype=np.uint8)
        self._check(self.lib.tfan_get_state(self._handle, buf.ctypes.data_as(_vp), buf.size))
        return buf

    def set_state(self, buf: np.ndarray):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(self.lib.tfan_set_state(self._handle, buf.ctypes.data_as(_vp), buf.size))

    def sync(self):
        self._check(self.lib.tfan_sync(self._handle))

    def export_state(self, out):
        """Write (phi, Qxx, Qxy, u_a, u_p) as float32 [7][ny][nx], or with the two density
        deviations as [9][ny][nx], into the device tensor out (the plane count is its
        shape's)."""
        planes = _exchange_planes(out, self.ny, self.nx)
        self._check(self.lib.tfan_export_state(self._handle, _vp(out.data_ptr()), out.numel() * 4, planes))

    def import_state(self, x, step: int):
        """Set phi, Q and equilibrium populations giving back the velocities of the
        device tensor x: [7][ny][nx] keeps the handle's densities, [9][ny][nx] takes its
        own."""
        planes = _exchange_planes(x, self.ny, self.nx)
        self._check(self.lib.tfan_import_state(self._handle, _vp(x.data_ptr()), x.numel() * 4, planes, int(step)))

    def step_count(self) -> int:
        return int(self.lib.tfan_step_count(self._handle))

    def kernel_timing(self, cap: int):
        self._check(self.lib.tfan_kernel_timing(self._handle, int(cap)))

    def set_tuning(self, collide_rows: int, fd_shape: int):
        """Launch shape (results are bitwise the same for every shape): collide_rows in
        {1, 2} rows of sites per thread ({11, 12}: on half-width tiles); fd_shape in {1, 2, 4} (one
        launch per sub-step), {16, 32, 162, 163} (blocked sub-steps, both fields per block) or
        {165, 166} (blocked, phi and Q in separate blocks, 40- or 32-row tiles).  tfan.h documents
        each shape."""
        self._check(self.lib.tfan_set_tuning(self._handle, int(collide_rows), int(fd_shape)))

    def get_tuning(self) -> tuple:
        c, f = ctypes.c_int32(), ctypes.c_int32()
        self._check(self.lib.tfan_get_tuning(self._handle, ctypes.byref(c), ctypes.byref(f)))
        return c.value, f.value

    def autotune(self, steps: int = 20) -> float:
        ms = ctypes.c_double()
        self._check(self.lib.tfan_autotune(self._handle, int(steps), ctypes.byref(ms)))
        return ms.value

    def kernel_times(self) -> dict:
        k = int(self.lib.tfan_kernel_count())
        ms = (ctypes.c_double * k)()
        cnt = (ctypes.c_int64 * k)()
        self._check(self.lib.tfan_kernel_times(self._handle, ms, cnt, k))
        return {self.lib.tfan_kernel_name(i).decode(): (ms[i], cnt[i]) for i in range(k)}

    def close(self):
        if getattr(self, "_handle", None) and self._handle.value:
            self.lib.tfan_destroy(self._handle)
            self._handle = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent simulations advanced together (one launch per phase for all)."""

    def __init__(self, params_list, device=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the solver runs only on the GPU")
        self.lib = load_library()
        self.params = [dict(p) for p in params_list]
        arr = (tfan_params * len(self.params))(*[make_params(p) for p in self.params])
        nbytes = int(self.lib.tfan_batch_workspace_bytes(arr, len(self.params)))
        if nbytes == 0:
            for p in self.params:
                check_params(p)
            raise TfanError(TFAN_EINVAL, "invalid batch")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        aligned = (self.workspace.data_ptr() + 255) // 256 * 256
        self._handle = _vp()
        with torch.cuda.device(self.device):
            rc = self.lib.tfan_batch_create(arr, len(self.params), _vp(aligned), nbytes,
                                            _vp(self.stream.cuda_stream), ctypes.byref(self._handle))
        if rc != TFAN_OK:
            raise TfanError(rc, self.lib.tfan_batch_last_error(None).decode())

    def _check(self, rc):
        if rc != TFAN_OK:
            raise TfanError(rc, self.lib.tfan_batch_last_error(self._handle).decode())

    def __len__(self):
        return len(self.params)

    def _member(self, member):
        if not 0 <= int(member) < len(self.params):
            raise TfanError(TFAN_EINVAL, f"member {member} out of range")
        return self.params[int(member)]

    def init_fields(self, member, phi, qxx, qxy, u_a=None, u_p=None):
        p = self._member(member)
        s = (int(p["ny"]), int(p["nx"]))
        arrs = [_f64(phi, s), _f64(qxx, s), _f64(qxy, s), _f64(u_a, (2,) + s), _f64(u_p, (2,) + s)]
        self._check(self.lib.tfan_batch_init_fields(self._handle, int(member), *[_ptr(a) for a in arrs]))

    def step(self, n: int = 1):
        self._check(self.lib.tfan_batch_step(self._handle, int(n)))

    def step_persistent(self, n: int = 1):
        """The same steps as step(), all in one persistent launch (n_sub <= 5)."""
        self._check(self.lib.tfan_batch_step_persistent(self._handle, int(n)))

    def persistent_blocks(self) -> int:
        return int(self.lib.tfan_batch_persistent_blocks(self._handle))

    def get_fields(self, member) -> dict:
        p = self._member(member)
        s = (int(p["ny"]), int(p["nx"]))
        out = dict(phi=np.empty(s), qxx=np.empty(s), qxy=np.empty(s), u_a=np.empty((2,) + s),
                   u_p=np.empty((2,) + s), rho_a=np.empty(s), rho_p=np.empty(s))
        self._check(self.lib.tfan_batch_get_fields(self._handle, int(member), *[
            _ptr(out[k]) for k in ("phi", "qxx", "qxy", "u_a", "u_p", "rho_a", "rho_p")]))
        return out

    def diagnostics(self, member) -> dict:
        d = tfan_diag()
        rc = self.lib.tfan_batch_diagnostics(self._handle, int(member), ctypes.byref(d))
        if rc not in (TFAN_OK, TFAN_ENONFINITE, TFAN_EUNSTABLE):
            self._check(rc)
        out = {name: getattr(d, name) for name, _ in tfan_diag._fields_}
        out["status"] = rc
        return out

    def set_tuning(self, collide_rows: int, fd_shape: int):
        self._check(self.lib.tfan_batch_set_tuning(self._handle, int(collide_rows), int(fd_shape)))

    def get_tuning(self) -> tuple:
        c, f = ctypes.c_int32(), ctypes.c_int32()
        self._check(self.lib.tfan_batch_get_tuning(self._handle, ctypes.byref(c), ctypes.byref(f)))
        return c.value, f.value

    def autotune(self, steps: int = 10) -> float:
        ms = ctypes.c_double()
        self._check(self.lib.tfan_batch_autotune(self._handle, int(steps), ctypes.byref(ms)))
        return ms.value

    def sync(self):
        self._check(self.lib.tfan_batch_sync(self._handle))

    def close(self):
        if getattr(self, "_handle", None) and self._handle.value:
            self.lib.tfan_batch_destroy(self._handle)
            self._handle = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Cnn:
    """The convolutional surrogate network (include/tfan_cnn.h) on one stream.

    batch samples of ny x nx sites per call; train reserves the backward-pass
    buffers.  States are float32 device tensors [B][7][ny][nx]."""

    def __init__(self, batch: int, ny: int, nx: int, train: bool = False, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the network runs only on the GPU")
        self.lib = load_library()
        self.batch, self.ny, self.nx, self.train = int(batch), int(ny), int(nx), bool(train)
        nbytes = int(self.lib.tfan_cnn_workspace_bytes(self.batch, self.ny, self.nx, int(self.train)))
        if nbytes == 0:
            raise TfanError(TFAN_EINVAL, "batch >= 1 and ny, nx positive multiples of 16 required")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        self.stream = torch.cuda.current_stream() if stream is None else stream
        aligned = (self.workspace.data_ptr() + 255) // 256 * 256
        self._handle = _vp()
        rc = self.lib.tfan_cnn_create(self.batch, self.ny, self.nx, int(self.train), _vp(aligned), nbytes,
                                      _vp(self.stream.cuda_stream), ctypes.byref(self._handle))
        if rc != TFAN_OK:
            raise TfanError(rc, self.lib.tfan_cnn_last_error(None).decode())

    def _check(self, rc):
        if rc != TFAN_OK:
            raise TfanError(rc, self.lib.tfan_cnn_last_error(self._handle).decode())

    @staticmethod
    def param_count() -> int:
        return int(load_library().tfan_cnn_param_count())

    def set_params(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float32).ravel()
        if th.size != self.param_count():
            raise TfanError(TFAN_EINVAL, f"expected {self.param_count()} parameters")
        self._check(self.lib.tfan_cnn_set_params(self._handle, th.ctypes.data_as(_P(ctypes.c_float))))

    def get_params(self) -> np.ndarray:
        th = np.empty(self.param_count(), dtype=np.float32)
        self._check(self.lib.tfan_cnn_get_params(self._handle, th.ctypes.data_as(_P(ctypes.c_float))))
        return th

    def set_scales(self, s_in, s_out):
        a = np.ascontiguousarray(s_in, dtype=np.float32).ravel()
        b = np.ascontiguousarray(s_out, dtype=np.float32).ravel()
        if a.size != 7 or b.size != 7:
            raise TfanError(TFAN_EINVAL, "7 input and 7 output scales required")
        self._check(self.lib.tfan_cnn_set_scales(self._handle, a.ctypes.data_as(_P(ctypes.c_float)),
                                                 b.ctypes.data_as(_P(ctypes.c_float))))

    def forward(self, x, out):
        _check_dev(x, (self.batch, 7, self.ny, self.nx))
        _check_dev(out, (self.batch, 7, self.ny, self.nx))
        self._check(self.lib.tfan_cnn_forward(self._handle, _vp(x.data_ptr()), _vp(out.data_ptr())))

    def _batch(self, X, T, idx):
        _check_dev(X, (7, self.ny, self.nx))
        _check_dev(T, (7, self.ny, self.nx))
        if X.shape != T.shape or X.dim() != 4:
            raise TfanError(TFAN_EINVAL, "X and T must be stacks [n][7][ny][nx] of equal size")
        ix = np.ascontiguousarray(idx, dtype=np.int32).ravel()
        if ix.size != self.batch:
            raise TfanError(TFAN_EINVAL, f"{self.batch} sample indices required")
        return ix

    def gradients(self, X, T, idx):
        """(loss, gradient vector) of the batch X[idx] -> T[idx]."""
        ix = self._batch(X, T, idx)
        g = np.empty(self.param_count(), dtype=np.float32)
        loss = ctypes.c_double()
        self._check(self.lib.tfan_cnn_gradients(self._handle, _vp(X.data_ptr()), _vp(T.data_ptr()), X.shape[0],
                                                ix.ctypes.data_as(_P(ctypes.c_int32)),
                                                g.ctypes.data_as(_P(ctypes.c_float)), ctypes.byref(loss)))
        return loss.value, g

    def train_step(self, X, T, idx, lr: float, want_loss: bool = True):
        ix = self._batch(X, T, idx)
        loss = ctypes.c_double()
        self._check(self.lib.tfan_cnn_train_step(self._handle, _vp(X.data_ptr()), _vp(T.data_ptr()), X.shape[0],
                                                 ix.ctypes.data_as(_P(ctypes.c_int32)), float(lr),
                                                 ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def compare(self, a, b) -> np.ndarray:
        """[7][2]: per channel sum (a - b)^2 and sum b^2."""
        _check_dev(a, (self.batch, 7, self.ny, self.nx))
        _check_dev(b, (self.batch, 7, self.ny, self.nx))
        out = np.empty(14)
        self._check(self.lib.tfan_cnn_compare(self._handle, _vp(a.data_ptr()), _vp(b.data_ptr()), _ptr(out)))
        return out.reshape(7, 2)

    def sync(self):
        self._check(self.lib.tfan_cnn_sync(self._handle))

    def close(self):
        if getattr(self, "_handle", None):
            self.lib.tfan_cnn_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Analysis:
    """On-device observables (include/tfan_analysis.h) of exported states
    [7][n][n] (float32 device tensors) on an n x n grid, n a power of two."""

    def __init__(self, n: int, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the analysis runs only on the GPU")
        self.lib = load_library()
        self.n = int(n)
        nbytes = int(self.lib.tfan_analysis_workspace_bytes(self.n))
        if nbytes == 0:
            raise TfanError(TFAN_EINVAL, "n must be a power of two in [8, 4096]")
        self.shells = int(self.lib.tfan_analysis_shells(self.n))
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        self.stream = torch.cuda.current_stream() if stream is None else stream
        aligned = (self.workspace.data_ptr() + 255) // 256 * 256
        self._handle = _vp()
        rc = self.lib.tfan_analysis_create(self.n, _vp(aligned), nbytes, _vp(self.stream.cuda_stream),
                                           ctypes.byref(self._handle))
        if rc != TFAN_OK:
            raise TfanError(rc, self.lib.tfan_analysis_last_error(None).decode())

    def _check(self, rc):
        if rc != TFAN_OK:
            raise TfanError(rc, self.lib.tfan_analysis_last_error(self._handle).decode())

    def _state(self, x):
        _check_dev(x, (7, self.n, self.n))
        return _vp(x.data_ptr())

    def spectra(self, x) -> dict:
        out = {k: np.empty(self.shells) for k in ("E", "W", "S", "count")}
        L = ctypes.c_double()
        self._check(self.lib.tfan_analysis_spectra(self._handle, self._state(x), _ptr(out["E"]), _ptr(out["W"]),
                                                   _ptr(out["S"]), _ptr(out["count"]), ctypes.byref(L)))
        out["L"] = L.value
        return out

    def correlations(self, x) -> dict:
        out = {k: np.empty(self.shells) for k in ("uu", "ww", "QQ", "count")}
        self._check(self.lib.tfan_analysis_correlations(self._handle, self._state(x), _ptr(out["uu"]),
                                                        _ptr(out["ww"]), _ptr(out["QQ"]), _ptr(out["count"])))
        return out

    def all(self, x) -> dict:
        """Spectra, L, correlations and defect counts of one state in one call (the
        forward transforms computed once); keys as spectra() and correlations(),
        plus "defects" = (plus, minus)."""
        out = {k: np.empty(self.shells) for k in ("E", "W", "S", "uu", "ww", "QQ", "count")}
        L, p, m = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.tfan_analysis_all(self._handle, self._state(x), _ptr(out["E"]), _ptr(out["W"]),
                                               _ptr(out["S"]), ctypes.byref(L), _ptr(out["uu"]), _ptr(out["ww"]),
                                               _ptr(out["QQ"]), _ptr(out["count"]), ctypes.byref(p),
                                               ctypes.byref(m)))
        out["L"] = L.value
        out["defects"] = (p.value, m.value)
        return out

    def overlaps(self, x0, x1) -> np.ndarray:
        out = np.empty(6)
        self._check(self.lib.tfan_analysis_overlaps(self._handle, self._state(x0), self._state(x1), _ptr(out)))
        return out

    def defects(self, x) -> tuple:
        p, m = ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.tfan_analysis_defects(self._handle, self._state(x), ctypes.byref(p), ctypes.byref(m)))
        return p.value, m.value

    def close(self):
        if getattr(self, "_handle", None):
            self.lib.tfan_analysis_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def analysis_overlaps_noalloc(x0, x1, stream=None) -> np.ndarray:
    """tfan_analysis_overlaps_noalloc: the six overlap means of two exported states
    [7][n][n] (float32 device tensors), computed without any device allocation."""
    import torch
    lib = load_library()
    _check_dev(x0)
    _check_dev(x1)
    n = int(x0.shape[-1])
    if tuple(x0.shape[-3:]) != (7, n, n) or tuple(x1.shape[-3:]) != (7, n, n):
        raise TfanError(TFAN_EINVAL, "expected two states of shape [7][n][n]")
    st = stream if stream is not None else torch.cuda.current_stream()
    out = np.empty(6)
    rc = lib.tfan_analysis_overlaps_noalloc(n, _vp(x0.data_ptr()), _vp(x1.data_ptr()), _ptr(out),
                                            _vp(st.cuda_stream))
    if rc != TFAN_OK:
        raise TfanError(rc, lib.tfan_analysis_noalloc_last_error().decode())
    return out
