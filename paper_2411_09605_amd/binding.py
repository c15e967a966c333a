"""ctypes binding of ``libpic.so`` (the C ABI in ``include/pic.h``).

Argument marshalling only: every step of the method runs in the library's HIP kernels.
PyTorch supplies device memory (tensors) and the HIP stream.  Importing this module
loads the library and raises if it has not been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpic.so")

PIC_OK, PIC_EINVAL, PIC_ENOMEM, PIC_EDEVICE, PIC_ESTATE, PIC_ENONFINITE, PIC_EUNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6
SCHEMES = {"esec2": 0, "esec1": 1, "emec_li": 2, "standard": 3, "emec_psatd": 4, "emec_lf": 5}
EM_SCHEMES = ("emec_li", 2, "emec_psatd", 4, "emec_lf", 5)
F_INIT_GAUSS, F_TRACK_IDS, F_INTERLEAVE, F_DETERMINISTIC, F_FILTER_RHO = 1, 2, 4, 8, 16
F_CHARGE_CONSERVING = 32
DEPOSIT_MODES = {"auto": 0, "lds_atomic": 1, "window": 2, "wave": 3, "lds_f64": 4}
ABI_VERSION = 1


class PicParams(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_int32), ("nv", ctypes.c_int32),
                ("scheme", ctypes.c_int32), ("shape_order", ctypes.c_int32),
                ("n_particles", ctypes.c_int64), ("n_cells", ctypes.c_int32),
                ("rebin_every", ctypes.c_int32), ("length", ctypes.c_double),
                ("dt", ctypes.c_double), ("c", ctypes.c_double),
                ("b_ext", ctypes.c_double * 3), ("flags", ctypes.c_uint32),
                ("block_threads", ctypes.c_int32), ("grid_blocks", ctypes.c_int32),
                ("deposit_mode", ctypes.c_int32), ("record_capacity", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class PicBuffers(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("v", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("id", ctypes.c_void_p), ("E", ctypes.c_void_p), ("B", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t)]


DIAG_DTYPE = np.dtype([("step", "i8"), ("time", "f8"), ("kinetic", "f8"), ("field_e", "f8"),
                       ("field_b", "f8"), ("total", "f8"), ("rel_energy_err", "f8"),
                       ("max_gamma_dev", "f8"), ("fallbacks", "i8"), ("fallbacks_total", "i8"),
                       ("nonfinite", "i4"), ("pad", "i4")])

# Every function declared in include/pic.h.
EXPORTS = ("pic_workspace_size", "pic_validate_params", "pic_init", "pic_step",
           "pic_diagnostics", "pic_sync_state", "pic_profile_enable", "pic_profile_read",
           "pic_launch_shape", "pic_destroy", "pic_strerror", "pic_last_error",
           "pic_run_static", "pic_state_size", "pic_save_state", "pic_load_state",
           "pic_check_inputs")
STATIC_SCRATCH_BYTES = 16 << 20
KERNEL_CLASSES = ("pass_a", "pass_b", "rebin")


class PicError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


def _load():
    # torch bundles the HIP runtime under the same soname; importing it first makes the
    # library bind to that one runtime, so torch's streams and pointers are valid here.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2411_09605_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(PicParams)
    vp = ctypes.c_void_p
    lib.pic_workspace_size.argtypes = [P]
    lib.pic_workspace_size.restype = ctypes.c_size_t
    lib.pic_validate_params.argtypes = [P]
    lib.pic_validate_params.restype = ctypes.c_int
    lib.pic_init.argtypes = [P, ctypes.POINTER(PicBuffers), vp, ctypes.POINTER(vp)]
    lib.pic_init.restype = ctypes.c_int
    lib.pic_step.argtypes = [vp, ctypes.c_int64]
    lib.pic_step.restype = ctypes.c_int
    lib.pic_diagnostics.argtypes = [vp, vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    lib.pic_diagnostics.restype = ctypes.c_int
    lib.pic_sync_state.argtypes = [vp]
    lib.pic_sync_state.restype = ctypes.c_int
    lib.pic_profile_enable.argtypes = [vp, ctypes.c_int]
    lib.pic_profile_enable.restype = ctypes.c_int
    lib.pic_profile_read.argtypes = [vp, vp, vp]
    lib.pic_profile_read.restype = ctypes.c_int
    lib.pic_launch_shape.argtypes = [vp, vp, vp, vp]
    lib.pic_launch_shape.restype = ctypes.c_int
    lib.pic_destroy.argtypes = [vp]
    lib.pic_destroy.restype = ctypes.c_int
    lib.pic_strerror.argtypes = [ctypes.c_int]
    lib.pic_strerror.restype = ctypes.c_char_p
    lib.pic_last_error.argtypes = [vp]
    lib.pic_last_error.restype = ctypes.c_char_p
    lib.pic_run_static.argtypes = [P, ctypes.POINTER(PicBuffers), vp, ctypes.c_int64, vp]
    lib.pic_run_static.restype = ctypes.c_int
    dp = ctypes.POINTER(ctypes.c_double)
    lib.pic_check_inputs.argtypes = [P, dp, dp, dp, dp, dp, ctypes.POINTER(ctypes.c_int64)]
    lib.pic_check_inputs.restype = ctypes.c_int
    lib.pic_state_size.argtypes = [vp]
    lib.pic_state_size.restype = ctypes.c_size_t
    lib.pic_save_state.argtypes = [vp, vp, ctypes.c_size_t]
    lib.pic_save_state.restype = ctypes.c_int
    lib.pic_load_state.argtypes = [vp, vp, ctypes.c_size_t]
    lib.pic_load_state.restype = ctypes.c_int
    return lib


lib = _load()


def make_params(nv: int, scheme, shape_order: int, n_particles: int, n_cells: int,
                length: float, dt: float, c: float = 1.0, b_ext=(0.0, 0.0, 0.0),
                init_gauss: bool = False, track_ids: bool = False, rebin_every: int = 0,
                block_threads: int = 0, grid_blocks: int = 0, deposit_mode="auto",
                record_capacity: int = 0, interleave: bool = False,
                deterministic: bool = False, filter_rho: bool = False,
                charge_conserving: bool = False) -> PicParams:
    p = PicParams()
    p.abi_version = ABI_VERSION
    p.nv, p.scheme, p.shape_order = nv, SCHEMES.get(scheme, scheme), shape_order
    p.n_particles, p.n_cells, p.rebin_every = n_particles, n_cells, rebin_every
    p.length, p.dt, p.c = length, dt, c
    for i in range(3):
        p.b_ext[i] = b_ext[i]
    p.flags = ((F_INIT_GAUSS if init_gauss else 0) | (F_TRACK_IDS if track_ids else 0)
               | (F_INTERLEAVE if interleave else 0) | (F_DETERMINISTIC if deterministic else 0)
               | (F_FILTER_RHO if filter_rho else 0)
               | (F_CHARGE_CONSERVING if charge_conserving else 0))
    p.block_threads, p.grid_blocks = block_threads, grid_blocks
    p.deposit_mode = DEPOSIT_MODES.get(deposit_mode, deposit_mode)
    p.record_capacity, p.reserved = record_capacity, 0
    return p


def validate(p: PicParams) -> int:
    return lib.pic_validate_params(ctypes.byref(p))


def check_inputs(p: PicParams, x, v, E, B=None, w=None):
    """pic_check_inputs on host arrays: (status, index of the first non-finite value or -1)."""
    def ptr(a):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=np.float64)
        keep.append(a)
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    keep = []
    bad = ctypes.c_int64()
    rc = lib.pic_check_inputs(ctypes.byref(p), ptr(x), ptr(v), ptr(w), ptr(E), ptr(B),
                              ctypes.byref(bad))
    return rc, bad.value


def workspace_size(p: PicParams) -> int:
    return lib.pic_workspace_size(ctypes.byref(p))


def last_error(ctx=None) -> str:
    return (lib.pic_last_error(ctx) or b"").decode()


def _check(rc: int, ctx=None):
    if rc != PIC_OK:
        raise PicError(rc, f"{lib.pic_strerror(rc).decode()}: {last_error(ctx)}")


class Pic:
    """One run bound to device tensors and a HIP stream.

    ``x`` [N_p], ``v`` [nv, N_p], ``E`` [3, N_g], ``B`` [2, N_g] (EM), ``w`` [N_p] or None,
    ``ids`` [N_p] int64 or None: contiguous float64/int64 CUDA tensors owned by the
    caller.  The workspace tensor is allocated here (uint8, 256-byte aligned)."""

    def __init__(self, params: PicParams, x, v, E, B=None, w=None, ids=None, stream=None):
        import torch
        self.torch = torch
        self.params = params
        for t in (x, v, E) + tuple(a for a in (B, w) if a is not None):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("x, v, E, B, w must be contiguous float64 CUDA tensors")
        n, ng, nv = params.n_particles, params.n_cells, params.nv
        if x.numel() != n or v.numel() != nv * n or E.numel() != 3 * ng:
            raise ValueError("array sizes do not match the parameters")
        if B is not None and B.numel() != 2 * ng:
            raise ValueError("B must hold 2 * n_cells values")
        if w is not None and w.numel() != n:
            raise ValueError("w must hold n_particles values")
        if ids is not None and (ids.dtype != torch.int64 or ids.numel() != n):
            raise ValueError("ids must be int64 with n_particles values")
        self.x, self.v, self.E, self.B, self.w, self.ids = x, v, E, B, w, ids
        nbytes = workspace_size(params)
        if nbytes == 0:
            _check(validate(params))
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=x.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(x.device)
        buf = PicBuffers()
        buf.x, buf.v, buf.E = x.data_ptr(), v.data_ptr(), E.data_ptr()
        buf.B = B.data_ptr() if B is not None else None
        buf.w = w.data_ptr() if w is not None else None
        buf.id = ids.data_ptr() if ids is not None else None
        buf.workspace, buf.workspace_bytes = aligned, nbytes
        self._buf = buf
        ctx = ctypes.c_void_p()
        _check(lib.pic_init(ctypes.byref(params), ctypes.byref(buf),
                            ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)))
        self.ctx = ctx
        self.records = []

    def step(self, n: int = 1):
        _check(lib.pic_step(self.ctx, n), self.ctx)

    def diagnostics(self, max_records: int = 1 << 20) -> np.ndarray:
        """Records written since the previous call (synchronises the stream)."""
        out = np.zeros(max_records, dtype=DIAG_DTYPE)
        nw = ctypes.c_int64()
        rc = lib.pic_diagnostics(self.ctx, out.ctypes.data, max_records, ctypes.byref(nw))
        if rc not in (PIC_OK, PIC_ENONFINITE):
            _check(rc, self.ctx)
        recs = out[:nw.value].copy()
        self.records.extend(recs)
        return recs

    def launch_shape(self) -> tuple:
        """(threads per workgroup, workgroups, particles per workgroup) of the passes."""
        t, g, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(lib.pic_launch_shape(self.ctx, ctypes.byref(t), ctypes.byref(g), ctypes.byref(c)),
               self.ctx)
        return t.value, g.value, c.value

    @property
    def block_threads(self) -> int:
        return self.launch_shape()[0]

    @property
    def grid_blocks(self) -> int:
        return self.launch_shape()[1]

    def profile(self, on: bool = True):
        """Turn HIP-event timing of each launch on or off."""
        _check(lib.pic_profile_enable(self.ctx, 1 if on else 0), self.ctx)

    def profile_read(self) -> dict:
        """{kernel class: (total ms, launches)} since the last read."""
        ms = np.zeros(len(KERNEL_CLASSES))
        n = np.zeros(len(KERNEL_CLASSES), dtype=np.int64)
        _check(lib.pic_profile_read(self.ctx, ms.ctypes.data, n.ctypes.data), self.ctx)
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNEL_CLASSES)}

    def sync_state(self):
        _check(lib.pic_sync_state(self.ctx), self.ctx)

    def save_state(self) -> np.ndarray:
        """The run's complete state (pic_save_state) as a uint8 host array."""
        n = int(lib.pic_state_size(self.ctx))
        if n == 0:
            raise PicError(PIC_ESTATE, "no state to save")
        buf = np.empty(n, dtype=np.uint8)
        _check(lib.pic_save_state(self.ctx, buf.ctypes.data, n), self.ctx)
        return buf

    def load_state(self, buf):
        """Continue from a state saved by ``save_state`` (pic_load_state)."""
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(lib.pic_load_state(self.ctx, buf.ctypes.data, buf.size), self.ctx)

    def state(self) -> dict:
        self.sync_state()
        d = dict(x=self.x.cpu().numpy(), v=self.v.reshape(self.params.nv, -1).cpu().numpy(),
                 E=self.E.reshape(3, -1).cpu().numpy())
        if self.B is not None:
            d["B"] = self.B.reshape(2, -1).cpu().numpy()
        if self.ids is not None:
            d["ids"] = self.ids.cpu().numpy()
        return d

    def destroy(self):
        if self.ctx:
            lib.pic_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    @classmethod
    def from_arrays(cls, nv, scheme, order, n_cells, length, dt, x, v, E0=None, B0=None,
                    w=None, c=1.0, b_ext=(0.0, 0.0, 0.0), init_gauss=False, ids=None,
                    track_ids=False, device="cuda", **knobs) -> "Pic":
        """Copy host arrays to the device and initialise a run.  ``track_ids`` without
        ``ids`` numbers the particles 0 .. N_p - 1."""
        import torch
        n = int(np.asarray(x).shape[0])
        cls.check_host_inputs(nv, scheme, order, n_cells, length, dt, x, v, E0=E0, B0=B0, w=w,
                              c=c, b_ext=b_ext, init_gauss=init_gauss, **knobs)
        if track_ids and ids is None:
            ids = np.arange(n, dtype=np.int64)
        f64 = dict(dtype=torch.float64, device=device)
        xt = torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)).to(**f64).contiguous()
        vt = torch.as_tensor(np.ascontiguousarray(v, dtype=np.float64).reshape(nv, n)).to(**f64).contiguous()
        Et = torch.zeros((3, n_cells), **f64)
        if E0 is not None:
            Et.copy_(torch.as_tensor(np.asarray(E0, dtype=np.float64).reshape(3, n_cells)))
        Bt = None
        if scheme in EM_SCHEMES:
            Bt = torch.zeros((2, n_cells), **f64)
            if B0 is not None:
                Bt.copy_(torch.as_tensor(np.asarray(B0, dtype=np.float64).reshape(2, n_cells)))
        wt = None if w is None else torch.as_tensor(np.ascontiguousarray(w, dtype=np.float64)).to(**f64)
        it = None
        if ids is not None:
            it = torch.as_tensor(np.ascontiguousarray(ids, dtype=np.int64)).to(device)
        p = make_params(nv, scheme, order, n, n_cells, length, dt, c=c, b_ext=b_ext,
                        init_gauss=init_gauss, track_ids=ids is not None, **knobs)
        return cls(p, xt, vt, Et, Bt, wt, it)

    @staticmethod
    def check_host_inputs(nv, scheme, order, n_cells, length, dt, x, v, E0=None, B0=None,
                          w=None, c=1.0, b_ext=(0.0, 0.0, 0.0), init_gauss=False, **knobs):
        """pic_check_inputs on the host arrays ``from_arrays`` would upload; raises
        PicError (PIC_ENONFINITE names the array and index)."""
        n = int(np.asarray(x).shape[0])
        p = make_params(nv, scheme, order, n, n_cells, length, dt, c=c, b_ext=b_ext,
                        init_gauss=init_gauss, **knobs)
        E = np.zeros((3, n_cells)) if E0 is None else E0
        B = (np.zeros((2, n_cells)) if B0 is None else B0) if scheme in EM_SCHEMES else B0
        rc, _ = check_inputs(p, x, v, E, B, w)
        _check(rc)

    @classmethod
    def from_workload(cls, wl, scheme: Optional[str] = None, device="cuda", **knobs) -> "Pic":
        """Build from any object with the fields of ``workloads.Workload``."""
        return cls.from_arrays(wl.nv, scheme or wl.scheme, wl.order, wl.n_cells, wl.length,
                               wl.dt, wl.x, wl.v, E0=wl.E0, B0=wl.B0, w=wl.w, c=wl.c,
                               b_ext=wl.b_ext, init_gauss=wl.init_gauss, device=device, **knobs)


def run_static(params: PicParams, x, v, E, B=None, w=None, ids=None, n_steps: int = 0,
               diag=None, stream=None) -> int:
    """``pic_run_static``: initialise and advance ``n_steps`` steps in one call, with the
    library's static workspace (no allocation in the library).  Tensors as for ``Pic``;
    ``diag`` is None or a CUDA tensor of at least ``DIAG_DTYPE.itemsize`` bytes that
    receives the newest step's record.  Asynchronous on ``stream``; returns the status
    (raises ``PicError`` on failure)."""
    import torch
    buf = PicBuffers()
    buf.x, buf.v, buf.E = x.data_ptr(), v.data_ptr(), E.data_ptr()
    buf.B = B.data_ptr() if B is not None else None
    buf.w = w.data_ptr() if w is not None else None
    buf.id = ids.data_ptr() if ids is not None else None
    buf.workspace, buf.workspace_bytes = None, 0
    if diag is not None and (not diag.is_cuda or diag.numel() * diag.element_size() < DIAG_DTYPE.itemsize):
        raise ValueError("diag must be a CUDA tensor of at least one pic_diag")
    s = stream if stream is not None else torch.cuda.current_stream(x.device)
    rc = lib.pic_run_static(ctypes.byref(params), ctypes.byref(buf), ctypes.c_void_p(s.cuda_stream),
                            int(n_steps), ctypes.c_void_p(diag.data_ptr()) if diag is not None else None)
    _check(rc)
    return rc


def diag_from_tensor(diag) -> np.ndarray:
    """The pic_diag a ``run_static`` call wrote into ``diag`` (synchronises)."""
    raw = diag.detach().reshape(-1).view(dtype=__import__("torch").uint8)[:DIAG_DTYPE.itemsize]
    return np.frombuffer(raw.cpu().numpy().tobytes(), dtype=DIAG_DTYPE)[0]


# ---------------------------------------------------------------- batched ensemble
class PicBatchParams(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_int32), ("n_runs", ctypes.c_int32),
                ("nv", ctypes.c_int32), ("scheme", ctypes.c_int32),
                ("shape_order", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("dt", ctypes.c_double), ("c", ctypes.c_double),
                ("b_ext", ctypes.c_double * 3),
                ("n_particles", ctypes.POINTER(ctypes.c_int64)),
                ("n_cells", ctypes.POINTER(ctypes.c_int32)),
                ("length", ctypes.POINTER(ctypes.c_double)),
                ("block_threads", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32), ("graph_steps", ctypes.c_int32),
                ("record_capacity", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class PicBatchBuffers(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("v", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("E", ctypes.c_void_p), ("B", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t)]


BATCH_EXPORTS = ("pic_batch_workspace_size", "pic_batch_init", "pic_batch_step",
                 "pic_batch_diagnostics", "pic_batch_destroy")


def _load_batch(L):
    vp = ctypes.c_void_p
    BP = ctypes.POINTER(PicBatchParams)
    L.pic_batch_workspace_size.argtypes = [BP]
    L.pic_batch_workspace_size.restype = ctypes.c_size_t
    L.pic_batch_init.argtypes = [BP, ctypes.POINTER(PicBatchBuffers), vp, ctypes.POINTER(vp)]
    L.pic_batch_init.restype = ctypes.c_int
    L.pic_batch_step.argtypes = [vp, ctypes.c_int64]
    L.pic_batch_step.restype = ctypes.c_int
    L.pic_batch_diagnostics.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int64,
                                        ctypes.POINTER(ctypes.c_int64)]
    L.pic_batch_diagnostics.restype = ctypes.c_int
    L.pic_batch_destroy.argtypes = [vp]
    L.pic_batch_destroy.restype = ctypes.c_int


_load_batch(lib)
EXPORTS = EXPORTS + BATCH_EXPORTS


def make_batch_params(nv, scheme, shape_order, n_particles, n_cells, length, dt, c=1.0,
                      b_ext=(0.0, 0.0, 0.0), init_gauss=True, block_threads=0, chunk=0,
                      grid_blocks=0, graph_steps=0, record_capacity=0) -> PicBatchParams:
    """A pic_batch_params; the per-run arrays are kept alive on the returned struct."""
    p = PicBatchParams()
    p._np = np.ascontiguousarray(n_particles, dtype=np.int64)
    p._ng = np.ascontiguousarray(n_cells, dtype=np.int32)
    p._len = np.ascontiguousarray(length, dtype=np.float64)
    if not (len(p._np) == len(p._ng) == len(p._len)):
        raise ValueError("per-run arrays differ in length")
    p.abi_version = ABI_VERSION
    p.n_runs = len(p._np)
    p.nv = nv
    p.scheme = SCHEMES[scheme] if isinstance(scheme, str) else scheme
    p.shape_order = shape_order
    p.flags = 1 if init_gauss else 0
    p.dt, p.c = dt, c
    for i in range(3):
        p.b_ext[i] = b_ext[i]
    p.n_particles = p._np.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    p.n_cells = p._ng.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    p.length = p._len.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p.block_threads, p.chunk, p.grid_blocks = block_threads, chunk, grid_blocks
    p.graph_steps, p.record_capacity, p.reserved = graph_steps, record_capacity, 0
    return p


def batch_workspace_size(p: PicBatchParams) -> int:
    return int(lib.pic_batch_workspace_size(ctypes.byref(p)))


def pack_runs(runs, device="cuda") -> dict:
    """Pack the runs' particles and fields into the batched layout on the device.

    Returns a dict of tensors (x, v, w or None, E, B or None) and host index arrays; a
    PicBatch built from it steps clones of the tensors, so one packing can serve several
    contexts (the autotuner, the benchmark)."""
    import torch
    r0 = runs[0]
    for r in runs:
        if (r.nv, r.scheme, r.order, r.dt, r.c, tuple(r.b_ext)) != \
                (r0.nv, r0.scheme, r0.order, r0.dt, r0.c, tuple(r0.b_ext)):
            raise ValueError("runs of a batch share nv, scheme, order, dt, c and b_ext")
    nv = r0.nv
    np_ = np.array([r.n_particles for r in runs], dtype=np.int64)
    ng_ = np.array([r.n_cells for r in runs], dtype=np.int32)
    len_ = np.array([r.length for r in runs], dtype=np.float64)
    poff = np.concatenate([[0], np.cumsum(np_)])
    goff = np.concatenate([[0], np.cumsum(ng_)])
    N, G = int(poff[-1]), int(goff[-1])
    f64 = dict(dtype=torch.float64, device=device)
    x = torch.empty(N, **f64)
    v = torch.empty((nv, N), **f64)
    for k, r in enumerate(runs):
        a, b = int(poff[k]), int(poff[k + 1])
        x[a:b] = torch.as_tensor(np.asarray(r.x, dtype=np.float64))
        v[:, a:b] = torch.as_tensor(np.asarray(r.v, dtype=np.float64).reshape(nv, -1))
    Eh = np.zeros(3 * G)
    Bh = np.zeros(2 * G)
    for k, r in enumerate(runs):
        g0, ng = int(goff[k]), int(ng_[k])
        if r.E0 is not None:
            Eh[3 * g0:3 * g0 + 3 * ng] = np.asarray(r.E0, dtype=np.float64).reshape(-1)
        if r.B0 is not None:
            Bh[2 * g0:2 * g0 + 2 * ng] = np.asarray(r.B0, dtype=np.float64).reshape(-1)
    w = None
    if any(r.w is not None for r in runs):
        w = torch.as_tensor(np.concatenate(
            [np.asarray(r.w, dtype=np.float64) if r.w is not None
             else np.full(r.n_particles, r.length / r.n_particles) for r in runs])).to(**f64)
    return dict(x=x, v=v, w=w, E=torch.as_tensor(Eh).to(**f64),
                B=torch.as_tensor(Bh).to(**f64) if r0.scheme in EM_SCHEMES else None,
                np=np_, ng=ng_, len=len_, poff=poff, goff=goff, nv=nv, r0=r0,
                init_gauss=all(r.init_gauss for r in runs))


class PicBatch:
    """Many independent runs advanced together (one persistent launch per pass).

    Built from a list of run descriptions with the fields of ``workloads.Workload`` that
    share nv, scheme, order, dt, c and b_ext (or from ``pack_runs`` of such a list).
    Particles are packed run after run."""

    def __init__(self, runs=None, device="cuda", block_threads=0, chunk=0, grid_blocks=0,
                 graph_steps=0, record_capacity=0, stream=None, packed=None):
        import torch
        self.torch = torch
        if packed is None:
            packed = pack_runs(runs, device)
            own = True
        else:
            own = False
        r0 = packed["r0"]
        self.nv = packed["nv"]
        self.np_, self.ng_, self.len_ = packed["np"], packed["ng"], packed["len"]
        self.poff, self.goff = packed["poff"], packed["goff"]
        self.nruns = len(self.np_)

        def mine(t):
            return None if t is None else (t if own else t.clone())
        self.x, self.v, self.w = mine(packed["x"]), mine(packed["v"]), packed["w"]
        self.E, self.B = mine(packed["E"]), mine(packed["B"])
        p = make_batch_params(r0.nv, r0.scheme, r0.order, self.np_, self.ng_, self.len_,
                              dt=r0.dt, c=r0.c, b_ext=r0.b_ext, init_gauss=packed["init_gauss"],
                              block_threads=block_threads, chunk=chunk,
                              grid_blocks=grid_blocks, graph_steps=graph_steps,
                              record_capacity=record_capacity)
        self.params = p
        nbytes = batch_workspace_size(p)
        if nbytes == 0:
            raise PicError(PIC_EINVAL, last_error())
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.x.device)
        aligned = (self.workspace.data_ptr() + 255) // 256 * 256
        # graph replay needs a stream other than the legacy default one
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.x.device)
        torch.cuda.synchronize(self.x.device)
        buf = PicBatchBuffers()
        buf.x, buf.v, buf.E = self.x.data_ptr(), self.v.data_ptr(), self.E.data_ptr()
        buf.B = self.B.data_ptr() if self.B is not None else None
        buf.w = self.w.data_ptr() if self.w is not None else None
        buf.workspace, buf.workspace_bytes = aligned, nbytes
        self._buf = buf
        ctx = ctypes.c_void_p()
        rc = lib.pic_batch_init(ctypes.byref(p), ctypes.byref(buf),
                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
        _check(rc)
        self.ctx = ctx

    @property
    def n_particles_total(self) -> int:
        return int(self.poff[-1])

    def step(self, n: int = 1):
        _check(lib.pic_batch_step(self.ctx, n))

    def diagnostics(self, run: int, max_records: int = 1 << 16) -> np.ndarray:
        out = np.zeros(max_records, dtype=DIAG_DTYPE)
        nw = ctypes.c_int64()
        rc = lib.pic_batch_diagnostics(self.ctx, run, out.ctypes.data, max_records, ctypes.byref(nw))
        if rc not in (PIC_OK, PIC_ENONFINITE):
            _check(rc)
        return out[:nw.value].copy()

    def state(self, run: int) -> dict:
        self.torch.cuda.synchronize()
        a, b = int(self.poff[run]), int(self.poff[run + 1])
        g0, ng = int(self.goff[run]), int(self.ng_[run])
        d = dict(x=self.x[a:b].cpu().numpy(), v=self.v[:, a:b].cpu().numpy(),
                 E=self.E[3 * g0:3 * g0 + 3 * ng].reshape(3, ng).cpu().numpy())
        if self.B is not None:
            d["B"] = self.B[2 * g0:2 * g0 + 2 * ng].reshape(2, ng).cpu().numpy()
        return d

    def destroy(self):
        if getattr(self, "ctx", None):
            lib.pic_batch_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


# --------------------------------------------------------------------- adjoint form
ADJ_MAX_MODES = 16


class PicAdjParams(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_int32), ("shape_order", ctypes.c_int32),
                ("n_particles", ctypes.c_int64), ("n_cells", ctypes.c_int32),
                ("n_steps", ctypes.c_int32), ("checkpoint_every", ctypes.c_int32),
                ("n_modes", ctypes.c_int32), ("length", ctypes.c_double),
                ("dt", ctypes.c_double), ("loss_weight", ctypes.c_double),
                ("k", ctypes.c_double * ADJ_MAX_MODES), ("block_threads", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32), ("reserved", ctypes.c_int32 * 2)]


class PicAdjBuffers(ctypes.Structure):
    _fields_ = [("u", ctypes.c_void_p), ("s", ctypes.c_void_p), ("g", ctypes.c_void_p),
                ("x", ctypes.c_void_p), ("v", ctypes.c_void_p), ("E", ctypes.c_void_p),
                ("loss", ctypes.c_void_p), ("grad", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t)]


ADJ_EXPORTS = ("pic_adj_workspace_size", "pic_adj_init", "pic_adj_forward", "pic_adj_backward",
               "pic_adj_records", "pic_adj_destroy")


def _load_adj(L):
    vp = ctypes.c_void_p
    AP = ctypes.POINTER(PicAdjParams)
    L.pic_adj_workspace_size.argtypes = [AP]
    L.pic_adj_workspace_size.restype = ctypes.c_size_t
    L.pic_adj_init.argtypes = [AP, ctypes.POINTER(PicAdjBuffers), vp, ctypes.POINTER(vp)]
    L.pic_adj_init.restype = ctypes.c_int
    L.pic_adj_forward.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.c_double,
                                  ctypes.c_double]
    L.pic_adj_forward.restype = ctypes.c_int
    L.pic_adj_backward.argtypes = [vp, ctypes.c_double]
    L.pic_adj_backward.restype = ctypes.c_int
    L.pic_adj_records.argtypes = [vp, vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    L.pic_adj_records.restype = ctypes.c_int
    L.pic_adj_destroy.argtypes = [vp]
    L.pic_adj_destroy.restype = ctypes.c_int


_load_adj(lib)
EXPORTS = EXPORTS + ADJ_EXPORTS


def make_adj_params(shape_order, n_particles, n_cells, length, dt, n_steps, checkpoint_every,
                    ks=(), loss_weight=None, block_threads=0, grid_blocks=0) -> PicAdjParams:
    p = PicAdjParams()
    p.abi_version = ABI_VERSION
    p.shape_order = shape_order
    p.n_particles, p.n_cells = n_particles, n_cells
    p.n_steps, p.checkpoint_every = n_steps, checkpoint_every
    if len(ks) > ADJ_MAX_MODES:
        raise ValueError(f"at most {ADJ_MAX_MODES} modes")
    p.n_modes = len(ks)
    p.length, p.dt = length, dt
    p.loss_weight = dt if loss_weight is None else loss_weight
    for m, k in enumerate(ks):
        p.k[m] = k
    p.block_threads, p.grid_blocks = block_threads, grid_blocks
    p.reserved[0] = p.reserved[1] = 0
    return p


def adj_workspace_size(p: PicAdjParams) -> int:
    return int(lib.pic_adj_workspace_size(ctypes.byref(p)))


class PicAdjoint:
    """Loss J = loss_weight * sum_{n=1..N} W_E^n of an ESEC2 1D-1V run started from the
    Gauss solve, and its gradient with respect to (alpha_1..alpha_M, v_beam, v_spread).

    ``u``, ``s``, ``g`` ([N_p]) are the uniforms of the inverse-CDF positions, the beam
    factors and the spread draws (numpy arrays or float64 CUDA tensors)."""

    def __init__(self, shape_order, n_cells, length, dt, n_steps, ks, u, s, g,
                 checkpoint_every=50, loss_weight=None, block_threads=0, grid_blocks=0,
                 device="cuda", stream=None):
        import torch
        self.torch = torch
        f64 = dict(dtype=torch.float64, device=device)

        def dev(a):
            t = a if isinstance(a, torch.Tensor) else torch.as_tensor(np.asarray(a, dtype=np.float64))
            return t.to(**f64).contiguous()
        self.u, self.s, self.g = dev(u), dev(s), dev(g)
        n = self.u.numel()
        if self.s.numel() != n or self.g.numel() != n:
            raise ValueError("u, s and g must have the same length")
        self.n_modes = len(ks)
        p = make_adj_params(shape_order, n, n_cells, length, dt, n_steps, checkpoint_every,
                            ks, loss_weight, block_threads, grid_blocks)
        self.params = p
        nbytes = adj_workspace_size(p)
        if nbytes == 0:
            raise PicError(PIC_EINVAL, last_error())
        self.x = torch.empty(n, **f64)
        self.v = torch.empty(n, **f64)
        self.E = torch.zeros(3 * n_cells, **f64)
        self.loss = torch.zeros(1, **f64)
        self.grad = torch.zeros(self.n_modes + 2, **f64)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        aligned = (self.workspace.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.x.device)
        torch.cuda.synchronize(self.x.device)
        b = PicAdjBuffers()
        b.u, b.s, b.g = self.u.data_ptr(), self.s.data_ptr(), self.g.data_ptr()
        b.x, b.v, b.E = self.x.data_ptr(), self.v.data_ptr(), self.E.data_ptr()
        b.loss, b.grad = self.loss.data_ptr(), self.grad.data_ptr()
        b.workspace, b.workspace_bytes = aligned, nbytes
        self._buf = b
        ctx = ctypes.c_void_p()
        _check(lib.pic_adj_init(ctypes.byref(p), ctypes.byref(b),
                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)))
        self.ctx = ctx
        # forward runs so far and the parameters of the newest one: pic_adj_backward
        # differentiates the newest forward run of the context
        self.forward_count = 0
        self.theta = None

    @classmethod
    def from_workload(cls, wl, checkpoint_every=50, **kw):
        """For a workload of ``workloads.adjoint_two_stream`` (its draws are in meta)."""
        m = wl.meta
        return cls(wl.order, wl.n_cells, wl.length, wl.dt, wl.steps, [k for k, _ in m["modes"]],
                   m["u"], m["sign"], m["g"], checkpoint_every=checkpoint_every, **kw)

    def forward(self, alpha, v_beam, v_spread, sync=True):
        a = np.ascontiguousarray(alpha, dtype=np.float64)
        if a.size != self.n_modes:
            raise ValueError("one amplitude per mode")
        rc = lib.pic_adj_forward(self.ctx, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 float(v_beam), float(v_spread))
        _check(rc)
        self.forward_count += 1
        self.theta = (a.copy(), float(v_beam), float(v_spread))
        if sync:
            self.stream.synchronize()
            return float(self.loss.cpu()[0])
        return None

    def backward(self, loss_bar=1.0, sync=True):
        _check(lib.pic_adj_backward(self.ctx, float(loss_bar)))
        if sync:
            self.stream.synchronize()
            return self.grad.cpu().numpy().copy()
        return None

    def records(self) -> np.ndarray:
        out = np.zeros(self.params.n_steps + 1, dtype=DIAG_DTYPE)
        nw = ctypes.c_int64()
        _check(lib.pic_adj_records(self.ctx, out.ctypes.data, out.size, ctypes.byref(nw)))
        return out[:nw.value]

    def destroy(self):
        if getattr(self, "ctx", None):
            lib.pic_adj_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _make_loss_function():
    import torch

    class TwoStreamLoss(torch.autograd.Function):
        """J(theta) with theta = (alpha_1..alpha_M, v_beam, v_spread) as a float64 tensor;
        the forward runs pic_adj_forward, the backward pic_adj_backward (checkpointed)."""

        @staticmethod
        def forward(ctx, theta, adj):
            th = theta.detach().to("cpu", torch.float64).numpy().copy()
            M = adj.n_modes
            J = adj.forward(th[:M], th[M], th[M + 1])
            ctx.adj = adj
            ctx.theta = th
            ctx.forward_count = adj.forward_count
            ctx.theta_device = theta.device
            return torch.tensor(J, dtype=torch.float64, device=theta.device)

        @staticmethod
        def backward(ctx, gJ):
            adj, th, M = ctx.adj, ctx.theta, ctx.adj.n_modes
            if adj.forward_count != ctx.forward_count:
                # another forward ran on the shared context since this one (a second loss,
                # a probe, a line search): its checkpoints are the other run's, so run
                # this loss's forward again before the reverse sweep
                adj.forward(th[:M], th[M], th[M + 1])
                ctx.forward_count = adj.forward_count
            g = adj.backward(float(gJ.detach().cpu()))
            return torch.as_tensor(g, dtype=torch.float64, device=ctx.theta_device), None

    return TwoStreamLoss


def two_stream_loss(theta, adj: PicAdjoint):
    """Differentiable J(theta) through the hand-written adjoint."""
    global _LOSS_FN
    if _LOSS_FN is None:
        _LOSS_FN = _make_loss_function()
    return _LOSS_FN.apply(theta, adj)


_LOSS_FN = None
