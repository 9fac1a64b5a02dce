"""MI355X (gfx950) solver for the two-fluid active-nematic mixture of arXiv 2511.00445.

The hot path is the HIP library libtfan.so (C ABI in include/tfan.h); this package
holds its ctypes binding, the build script and seeded workload generators.
"""
from .binding import (Analysis, Batch, Cnn, Sim, TfanError, check_params, load_library, workspace_bytes,  # noqa: F401
                      TFAN_OK, TFAN_EINVAL, TFAN_ENOMEM, TFAN_EHIP, TFAN_ENONFINITE, TFAN_EUNSTABLE)

__all__ = ["Analysis", "Batch", "Cnn", "Sim", "TfanError", "check_params", "load_library", "workspace_bytes"]
