"""MI355X (gfx950) library for the explicit energy-conserving particle-in-cell step of
Ricketson & Hu.  The step runs in hand-written HIP kernels behind the C ABI of
``include/pic.h``; this package is the thin Python binding over it."""
from .binding import (  # noqa: F401
    Pic, PicBatch, pack_runs, PicAdjoint, two_stream_loss, PicError, PicParams, make_params, validate, workspace_size, last_error,
    DIAG_DTYPE, EXPORTS, LIB_PATH, run_static, diag_from_tensor, STATIC_SCRATCH_BYTES,
)
