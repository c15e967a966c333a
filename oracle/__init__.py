"""ctypes front end of the FP64 CPU oracle (``pic_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The oracle is the independent reference the GPU library is
checked against.  Only the test suite, the package smoke check and the benchmark's
CPU-baseline leg may import it; the library itself never does.  It shares no code with
the GPU path.  Pins that tie it to the paper live in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pic_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SCHEMES = {"esec2": 0, "esec1": 1, "emec_li": 2, "emec_psatd": 4, "emec_lf": 5}


class OCfg(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int32), ("scheme", ctypes.c_int32),
                ("order", ctypes.c_int32), ("n_cells", ctypes.c_int32),
                ("n_particles", ctypes.c_int64), ("length", ctypes.c_double),
                ("dt", ctypes.c_double), ("c", ctypes.c_double),
                ("b_ext", ctypes.c_double * 3), ("cc", ctypes.c_int32), ("pad", ctypes.c_int32)]


class ODiag(ctypes.Structure):
    _fields_ = [("kinetic", ctypes.c_double), ("field_e", ctypes.c_double),
                ("field_b", ctypes.c_double), ("total", ctypes.c_double),
                ("max_gamma_dev", ctypes.c_double), ("fallbacks", ctypes.c_int64),
                ("nonfinite", ctypes.c_int32), ("pad", ctypes.c_int32)]


DIAG_DTYPE = np.dtype([("kinetic", "f8"), ("field_e", "f8"), ("field_b", "f8"),
                       ("total", "f8"), ("max_gamma_dev", "f8"), ("fallbacks", "i8"),
                       ("nonfinite", "i4"), ("pad", "i4")])


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)
        L.oracle_run.argtypes = [ctypes.POINTER(OCfg), dp, dp, dp, dp, dp, ctypes.c_int64,
                                 ctypes.c_int, ctypes.c_void_p]
        L.oracle_run.restype = ctypes.c_int
        L.oracle_run_gamma.argtypes = L.oracle_run.argtypes + [dp]
        L.oracle_run_gamma.restype = ctypes.c_int
        L.oracle_check.argtypes = [ctypes.POINTER(OCfg)]
        L.oracle_stencil.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_int, ip, dp]
        L.oracle_stencil.restype = ctypes.c_int
        L.oracle_deposit.argtypes = [ctypes.c_int, ctypes.c_int64, dp, dp, dp, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_double, dp]
        L.oracle_gather.argtypes = [ctypes.c_int, ctypes.c_int64, dp, dp, ctypes.c_int,
                                    ctypes.c_double, ctypes.c_double, dp]
        L.oracle_gauss.argtypes = [ctypes.c_int, ctypes.c_int64, dp, dp, ctypes.c_int,
                                   ctypes.c_double, dp]
        L.oracle_cn_solve.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp]
        L.oracle_rho_cc.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_int, ctypes.c_double, dp]
        L.oracle_deposit_cc.argtypes = [ctypes.c_int64, dp, dp, dp, dp, ctypes.c_int,
                                        ctypes.c_double, dp]
        L.oracle_energy.argtypes = [ctypes.POINTER(OCfg), dp, dp, dp, dp, ctypes.c_void_p]
        L.oracle_psatd.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                   dp, dp, dp, dp, dp, dp]
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_cfg(nv, scheme, order, n_cells, n_particles, length, dt, c=1.0, b_ext=(0, 0, 0),
             charge_conserving=False):
    cfg = OCfg()
    cfg.cc = 1 if charge_conserving else 0
    cfg.nv, cfg.scheme, cfg.order, cfg.n_cells = nv, SCHEMES.get(scheme, scheme), order, n_cells
    cfg.n_particles, cfg.length, cfg.dt, cfg.c = n_particles, length, dt, c
    for i in range(3):
        cfg.b_ext[i] = b_ext[i]
    return cfg


class State:
    """Host arrays of one run, in the layout the oracle uses (SoA FP64)."""

    def __init__(self, wl, scheme: Optional[str] = None, charge_conserving: bool = False):
        self.cfg = make_cfg(wl.nv, scheme or wl.scheme, wl.order, wl.n_cells,
                            wl.n_particles, wl.length, wl.dt, wl.c, wl.b_ext,
                            charge_conserving=charge_conserving)
        self.x = np.ascontiguousarray(wl.x, dtype=np.float64).copy()
        self.v = np.ascontiguousarray(wl.v, dtype=np.float64).reshape(wl.nv, -1).copy()
        self.w = None if wl.w is None else np.ascontiguousarray(wl.w, dtype=np.float64).copy()
        self.E = np.zeros((3, wl.n_cells)) if wl.E0 is None else \
            np.ascontiguousarray(wl.E0, dtype=np.float64).reshape(3, -1).copy()
        self.B = np.zeros((2, wl.n_cells)) if wl.B0 is None else \
            np.ascontiguousarray(wl.B0, dtype=np.float64).reshape(2, -1).copy()
        self.pending_gauss = bool(wl.init_gauss)
        self.records = []

    def run(self, nsteps: int, gamma_out: Optional[np.ndarray] = None) -> np.ndarray:
        """Advance ``nsteps``; returns the records (initial state first).  ``gamma_out``
        ([N_p]) receives Gamma of the last step, NaN where the fallback was taken."""
        rec = np.zeros(nsteps + 1, dtype=DIAG_DTYPE)
        rc = lib().oracle_run_gamma(ctypes.byref(self.cfg), _p(self.x), _p(self.v),
                                    _p(self.w), _p(self.E), _p(self.B), nsteps,
                                    int(self.pending_gauss), rec.ctypes.data, _p(gamma_out))
        if rc != 0:
            raise ValueError("oracle rejected the configuration")
        self.pending_gauss = False
        if not self.records:
            self.records.append(rec[0])
        self.records.extend(rec[1:])
        return rec


def stencil(order: int, pos: float, h: float, ng: int, shift: float = 0.0):
    idx = np.zeros(4, dtype=np.int64)
    wt = np.zeros(4)
    n = lib().oracle_stencil(order, pos, h, shift, ng,
                             idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _p(wt))
    return idx[:n].copy(), wt[:n].copy()


def deposit(order, x, w, u, ng, h, shift=0.0):
    x = np.ascontiguousarray(x, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(ng)
    lib().oracle_deposit(order, x.size, _p(x), _p(w), _p(u), ng, h, shift, _p(out))
    return out


def gather(order, x, field, h, shift=0.0):
    x = np.ascontiguousarray(x, dtype=np.float64)
    field = np.ascontiguousarray(field, dtype=np.float64)
    out = np.zeros(x.size)
    lib().oracle_gather(order, x.size, _p(x), _p(field), field.size, h, shift, _p(out))
    return out


def gauss(order, x, w, ng, length):
    x = np.ascontiguousarray(x, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    E = np.zeros(ng)
    lib().oracle_gauss(order, x.size, _p(x), _p(w), ng, length, _p(E))
    return E


def rho_cc(x, w, ng, h):
    """Charge density on the nodes with the quadratic B-spline (section 3.5's S')."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    rho = np.zeros(ng)
    lib().oracle_rho_cc(x.size, _p(x), _p(w), ng, h, _p(rho))
    return rho


def deposit_cc(x0, x1, w, u, ng, h):
    """Charge-conserving current on the half nodes from the paths x0 -> x1 (section 3.5)."""
    x0, x1, w, u = (np.ascontiguousarray(a, dtype=np.float64) for a in (x0, x1, w, u))
    out = np.zeros(ng)
    lib().oracle_deposit_cc(x0.size, _p(x0), _p(x1), _p(w), _p(u), ng, h, _p(out))
    return out


def cn_solve(ng, h, s, r):
    r = np.ascontiguousarray(r, dtype=np.float64)
    y = np.zeros(ng)
    lib().oracle_cn_solve(ng, h, s, _p(r), _p(y))
    return y


def psatd(ng, L, c, tau, E, B, J, average=True):
    """One PSATD field update over tau with the current held fixed: (E', B', <E> or None)."""
    E = np.ascontiguousarray(E, dtype=np.float64).reshape(3, ng)
    B = np.ascontiguousarray(B, dtype=np.float64).reshape(2, ng)
    J = np.ascontiguousarray(J, dtype=np.float64).reshape(3, ng)
    Eo, Bo, Ea = np.zeros((3, ng)), np.zeros((2, ng)), np.zeros((3, ng))
    lib().oracle_psatd(ng, L, c, tau, _p(E), _p(B), _p(J), _p(Eo), _p(Bo), _p(Ea) if average else None)
    return Eo, Bo, (Ea if average else None)


def energy(state: State) -> np.void:
    rec = np.zeros(1, dtype=DIAG_DTYPE)
    lib().oracle_energy(ctypes.byref(state.cfg), _p(state.v), _p(state.w), _p(state.E),
                        _p(state.B), rec.ctypes.data)
    return rec[0]


# ------------------------------------------------ standard explicit PIC (comparison)
def _std_sig():
    L = lib()
    if not getattr(L, "_std_ready", False):
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_std_run.argtypes = [ctypes.POINTER(OCfg), dp, dp, dp, dp, ctypes.c_int64,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
        L.oracle_std_run.restype = ctypes.c_int
        L.oracle_binomial.argtypes = [ctypes.c_int, dp, dp]
        L._std_ready = True
    return L


class StdState:
    """A run of the standard explicit PIC scheme (Vlasov-Poisson, symmetric leapfrog/Boris,
    section 5's comparison scheme) in the oracle; same host layout as ``State``.  E holds
    the newest half-step field E^{n-1/2} (E^0 before the first step); ``records`` the
    initial record and one per step."""

    def __init__(self, wl, filter_rho: bool = False):
        self.cfg = make_cfg(wl.nv, "esec2", wl.order, wl.n_cells, wl.n_particles, wl.length,
                            wl.dt, wl.c, wl.b_ext)
        self.x = np.ascontiguousarray(wl.x, dtype=np.float64).copy()
        self.v = np.ascontiguousarray(wl.v, dtype=np.float64).reshape(wl.nv, -1).copy()
        self.w = None if wl.w is None else np.ascontiguousarray(wl.w, dtype=np.float64).copy()
        self.E = np.zeros((3, wl.n_cells))
        self.B = np.zeros((2, wl.n_cells))
        self.filter = bool(filter_rho)
        self.records = []

    def run(self, nsteps: int) -> np.ndarray:
        """Advance ``nsteps``; returns the records (the current state's first)."""
        first = not self.records
        rec = np.zeros(nsteps + 1, dtype=DIAG_DTYPE)
        e = np.ascontiguousarray(self.E[0]).copy()
        rc = _std_sig().oracle_std_run(ctypes.byref(self.cfg), _p(self.x), _p(self.v),
                                       _p(self.w), _p(e), nsteps, int(self.filter), int(first),
                                       rec.ctypes.data)
        if rc != 0:
            raise ValueError("oracle rejected the configuration")
        self.E[0] = e
        if first:
            self.records.append(rec[0])
        else:
            rec[0] = self.records[-1]
        self.records.extend(rec[1:])
        return rec


def binomial(f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    _std_sig().oracle_binomial(f.size, _p(f), _p(out))
    return out


# ------------------------------------------------------------ tangent-linear derivative
def _tlm_sig():
    L = lib()
    if not getattr(L, "_tlm_ready", False):
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_tlm_run.argtypes = [ctypes.POINTER(OCfg), dp, dp, dp, dp, ctypes.c_int64,
                                     ctypes.c_int, ctypes.c_double, ctypes.c_int, dp, dp, dp,
                                     dp, dp, ctypes.c_void_p]
        L.oracle_tlm_run.restype = ctypes.c_int
        L.oracle_gauss_rho.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
        L._tlm_ready = True
    return L


def tlm_run(wl, nsteps: int, dx, dv, loss_weight: float, dE=None):
    """Forward-mode derivative of an ESEC2 1D-1V run of ``nsteps`` steps.

    ``dx``, ``dv``: [K, N_p] tangent directions of the initial positions and velocities;
    ``dE`` ([K, N_g]) only when the workload does not start from the Gauss solve.  The
    loss is ``loss_weight * sum_{n=1..N} W_E^n``.  Returns a dict with the loss ``J``,
    ``dJ`` [K], the final state (``x``, ``v``, ``E``), the final tangents (``dx``, ``dv``,
    ``dE``) and the records."""
    K = int(np.asarray(dx).shape[0]) if np.asarray(dx).ndim == 2 else 0
    n, ng = wl.n_particles, wl.n_cells
    cfg = make_cfg(1, "esec2", wl.order, ng, n, wl.length, wl.dt)
    x = np.ascontiguousarray(wl.x, dtype=np.float64).copy()
    v = np.ascontiguousarray(wl.v, dtype=np.float64).reshape(-1).copy()
    E = np.zeros(ng) if wl.E0 is None else \
        np.ascontiguousarray(np.asarray(wl.E0, dtype=np.float64).reshape(3, -1)[0]).copy()
    tx = np.ascontiguousarray(np.asarray(dx, dtype=np.float64).reshape(K, n)).copy()
    tv = np.ascontiguousarray(np.asarray(dv, dtype=np.float64).reshape(K, n)).copy()
    tE = np.zeros((K, ng)) if dE is None else \
        np.ascontiguousarray(np.asarray(dE, dtype=np.float64).reshape(K, ng)).copy()
    J = ctypes.c_double()
    dJ = np.zeros(max(K, 1))
    rec = np.zeros(nsteps + 1, dtype=DIAG_DTYPE)
    w = None if wl.w is None else np.ascontiguousarray(wl.w, dtype=np.float64).copy()
    rc = _tlm_sig().oracle_tlm_run(ctypes.byref(cfg), _p(x), _p(v), _p(w), _p(E), nsteps,
                                   int(wl.init_gauss), loss_weight, K, _p(tx), _p(tv), _p(tE),
                                   ctypes.cast(ctypes.byref(J), ctypes.POINTER(ctypes.c_double)),
                                   _p(dJ), rec.ctypes.data)
    if rc != 0:
        raise ValueError("tangent-linear run supports ESEC2 1D-1V only")
    return dict(J=J.value, dJ=dJ[:K], x=x, v=v, E=E, dx=tx, dv=tv, dE=tE, records=rec)


def density_mode_tangents(x, modes):
    """Derivative of inverse-CDF positions with respect to each mode amplitude.

    The positions solve F(x) = x + sum_j (alpha_j / k_j) sin(k_j x) = u L for the
    density 1 + sum_j alpha_j cos(k_j x); differentiating that identity at fixed u gives
    dx / d alpha_m = -sin(k_m x) / (k_m (1 + sum_j alpha_j cos(k_j x)))."""
    x = np.asarray(x, dtype=np.float64)
    dens = np.ones_like(x)
    for k, a in modes:
        dens = dens + a * np.cos(k * x)
    return np.stack([-np.sin(k * x) / (k * dens) for k, _ in modes])


def two_stream_gradient(wl, nsteps: int):
    """Reference gradient of J = dt sum_{n=1..N} W_E^n with respect to the mode
    amplitudes, the beam speed and the beam spread of a two-stream workload built by
    ``workloads.adjoint_two_stream`` (velocities v_b s_p + v_spread g_p): one
    tangent-linear run with one direction per parameter."""
    modes = wl.meta["modes"]
    n = wl.n_particles
    sign = np.asarray(wl.meta["sign"], dtype=np.float64)
    g = np.asarray(wl.meta["g"], dtype=np.float64)
    K = len(modes) + 2
    dx = np.zeros((K, n))
    dv = np.zeros((K, n))
    dx[:len(modes)] = density_mode_tangents(wl.x, modes)
    dv[len(modes)] = sign
    dv[len(modes) + 1] = g
    out = tlm_run(wl, nsteps, dx, dv, wl.dt)
    return out["J"], out["dJ"], out
