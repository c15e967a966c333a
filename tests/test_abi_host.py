"""Host-only checks of the C ABI (no GPU): the library loads, exports every function
declared in include/pic.h, and validates parameters without touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "pic.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pic_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    import paper_2411_09605_amd as P
    lib = ctypes.CDLL(P.LIB_PATH)
    names = _declared()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(P.EXPORTS) == names


def test_binding_requires_the_library(tmp_path):
    """Without the built library the package refuses to import (no fallback path)."""
    import shutil
    import subprocess
    import sys
    src = os.path.join(ROOT, "paper_2411_09605_amd")
    dst = tmp_path / "paper_2411_09605_amd"
    shutil.copytree(src, dst, ignore=shutil.ignore_patterns("*.so", "*.so.*", "__pycache__"))
    code = ("import sys; sys.path.insert(0, sys.argv[1])\n"
            "try:\n    import paper_2411_09605_amd\nexcept ImportError as e:\n"
            "    print('ImportError:', e); sys.exit(3)\n"
            "sys.exit(0)\n")
    r = subprocess.run([sys.executable, "-c", code, str(tmp_path)], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 3, (r.returncode, r.stdout, r.stderr)
    assert "libpic.so is missing" in r.stdout


def _good(**kw):
    import paper_2411_09605_amd as P
    base = dict(nv=1, scheme="esec2", shape_order=2, n_particles=1000, n_cells=64,
                length=10.0, dt=0.1)
    base.update(kw)
    return P.make_params(**base)


def test_validation_accepts_and_sizes():
    import paper_2411_09605_amd as P
    for kw in [{}, dict(scheme="esec1"), dict(nv=3, scheme="emec_li", n_cells=256),
               dict(nv=3, b_ext=(1.0, 0.0, 0.0)), dict(shape_order=1, n_cells=3),
               dict(n_particles=1), dict(block_threads=1024, grid_blocks=8192),
               dict(rebin_every=10), dict(rebin_every=1, deposit_mode="lds_atomic"),
               dict(deposit_mode="window"), dict(rebin_every=8, deposit_mode="wave"),
               dict(deterministic=True), dict(deterministic=True, deposit_mode="lds_atomic"),
               dict(nv=3, scheme="emec_li", n_cells=256, deterministic=True),
               dict(scheme="standard", init_gauss=True),
               dict(scheme="standard", init_gauss=True, filter_rho=True, nv=3),
               dict(scheme="standard", init_gauss=True, deterministic=True),
               dict(nv=3, scheme="emec_psatd", n_cells=256),
               dict(nv=3, scheme="emec_psatd", n_cells=3, shape_order=1),
               dict(nv=3, scheme="emec_psatd", n_cells=256, deterministic=True),
               dict(nv=3, scheme="emec_lf", n_cells=256, dt=0.039),
               dict(nv=3, scheme="emec_lf", n_cells=100, length=10.0, dt=0.1, c=1.0),
               dict(shape_order=1, charge_conserving=True, init_gauss=True),
               dict(shape_order=1, nv=3, charge_conserving=True, deposit_mode="lds_f64"),
               dict(shape_order=1, charge_conserving=True, deterministic=True)]:
        p = _good(**kw)
        assert P.validate(p) == 0, (kw, P.last_error())
        assert P.workspace_size(p) > 0


def test_validation_lds_limits():
    """The largest grids the particle passes fit in LDS (160 KB per workgroup, less 1 KB
    for the kernels' static LDS)."""
    import paper_2411_09605_amd as P
    for kw in [dict(n_cells=1842), dict(shape_order=1, n_cells=2254),
               dict(nv=3, scheme="emec_li", n_cells=697),
               dict(nv=3, scheme="emec_psatd", n_cells=697)]:
        assert P.validate(_good(**kw)) == 0, (kw, P.last_error())


@pytest.mark.parametrize("kw,code", [
    (dict(nv=2), -1), (dict(scheme=7), -1), (dict(nv=1, scheme="emec_li"), -1),
    (dict(shape_order=3), -1), (dict(n_particles=0), -1), (dict(n_cells=4), -1),
    (dict(shape_order=1, n_cells=2), -1), (dict(length=0.0), -1), (dict(dt=-1.0), -1),
    (dict(dt=float("nan")), -1), (dict(nv=3, scheme="emec_li", c=0.0), -1),
    (dict(nv=3, b_ext=(float("inf"), 0, 0)), -1), (dict(block_threads=100), -1),
    (dict(grid_blocks=100000), -1), (dict(deposit_mode=9), -1), (dict(rebin_every=-1), -1),
    (dict(n_cells=100000), -6), (dict(nv=3, scheme="emec_li", n_cells=4096), -6),
    # 159 KB of dynamic LDS per workgroup: quadratic ES pass B needs 11 N_g + 80 doubles,
    # EM 29 N_g + 128
    (dict(n_cells=1843), -6), (dict(nv=3, scheme="emec_li", n_cells=698), -6),
    (dict(shape_order=1, n_cells=2255), -6),
    (dict(interleave=True, rebin_every=5), -1),
    (dict(deterministic=True, rebin_every=5), -1),
    (dict(deterministic=True, deposit_mode="window"), -1),
    (dict(deterministic=True, deposit_mode="lds_f64"), -1),
    (dict(scheme="standard"), -1),                        # needs PIC_F_INIT_GAUSS
    (dict(filter_rho=True, init_gauss=True), -1),         # filter: standard scheme only
    (dict(scheme=5), -1), (dict(nv=1, scheme="emec_psatd"), -1),
    (dict(nv=3, scheme="emec_psatd", c=0.0), -1), (dict(nv=3, scheme="emec_psatd", c=float("inf")), -1),
    (dict(nv=3, scheme="emec_psatd", n_cells=698), -6),
    (dict(nv=3, scheme="emec_psatd", filter_rho=True), -1),
    (dict(nv=1, scheme="emec_lf"), -1), (dict(nv=3, scheme="emec_lf", c=0.0), -1),
    (dict(nv=3, scheme="emec_lf", n_cells=256, dt=0.05), -1),    # c dt > h: unstable leapfrog
    (dict(scheme=6), -1),
    (dict(charge_conserving=True), -1),                               # quadratic shapes
    (dict(shape_order=1, scheme="esec1", charge_conserving=True), -1),
    (dict(shape_order=1, nv=3, scheme="emec_li", charge_conserving=True), -1),
    (dict(shape_order=1, charge_conserving=True, rebin_every=4), -1),
    (dict(shape_order=1, charge_conserving=True, deposit_mode="window"), -1),
])
def test_validation_rejects(kw, code):
    import paper_2411_09605_amd as P
    p = _good(**kw)
    assert P.validate(p) == code, P.last_error()
    assert P.last_error()
    assert P.workspace_size(p) == 0


def test_rebin_workspace_is_larger():
    import paper_2411_09605_amd as P
    a = P.workspace_size(_good(n_particles=100_000))
    b = P.workspace_size(_good(n_particles=100_000, rebin_every=5))
    assert b >= a + 100_000 * 16


def test_abi_version_and_reserved_checked():
    import paper_2411_09605_amd as P
    p = _good()
    p.abi_version = 99
    assert P.validate(p) == -1
    p = _good()
    p.reserved = 1
    assert P.validate(p) == -1


def test_strerror_and_null_handling():
    import paper_2411_09605_amd as P
    lib = P.binding.lib
    assert lib.pic_strerror(0) == b"ok"
    assert lib.pic_strerror(-6) == b"unsupported configuration"
    assert lib.pic_validate_params(None) == -1
    assert lib.pic_step(None, 1) == -4
    assert lib.pic_destroy(None) == -4
    out = ctypes.c_void_p()
    assert lib.pic_init(None, None, None, ctypes.byref(out)) == -1


def _batch(**kw):
    import paper_2411_09605_amd.binding as B
    base = dict(nv=1, scheme="esec2", shape_order=1, n_particles=[1000, 50, 70000],
                n_cells=[64, 3, 512], length=[10.0, 3.0, 20.0], dt=0.1)
    base.update(kw)
    return B.make_batch_params(**base)


def test_batch_validation_accepts_and_sizes():
    import paper_2411_09605_amd.binding as B
    for kw in [{}, dict(shape_order=2, n_cells=[64, 5, 512]), dict(block_threads=64, chunk=128),
               dict(nv=3, scheme="emec_li", n_cells=[64, 5, 256]), dict(graph_steps=8),
               dict(n_particles=[1], n_cells=[8], length=[1.0])]:
        p = _batch(**kw)
        assert B.batch_workspace_size(p) > 0, (kw, B.last_error())
    # more work items, more workspace
    assert B.batch_workspace_size(_batch(chunk=256)) > B.batch_workspace_size(_batch())


@pytest.mark.parametrize("kw", [
    dict(n_particles=[], n_cells=[], length=[]), dict(n_cells=[64, 2, 512]),
    dict(n_particles=[1000, 0, 5]), dict(length=[10.0, -1.0, 1.0]), dict(chunk=100),
    dict(block_threads=96), dict(graph_steps=-1), dict(nv=1, scheme="emec_li"),
    dict(n_cells=[64, 3, 100000]), dict(dt=float("inf")), dict(scheme="standard"),
    dict(nv=3, scheme="emec_psatd"), dict(nv=3, scheme="emec_lf"),
])
def test_batch_validation_rejects(kw):
    import paper_2411_09605_amd.binding as B
    p = _batch(**kw)
    assert B.batch_workspace_size(p) == 0
    assert B.last_error()


def test_batch_null_handling():
    import paper_2411_09605_amd.binding as B
    lib = B.lib
    assert lib.pic_batch_step(None, 1) == -4
    assert lib.pic_batch_destroy(None) == -4
    assert lib.pic_batch_workspace_size(None) == 0


def _adj(**kw):
    import paper_2411_09605_amd.binding as B
    base = dict(shape_order=2, n_particles=10_000, n_cells=64, length=31.4, dt=0.05,
                n_steps=100, checkpoint_every=10, ks=[0.2 * m for m in range(1, 9)])
    base.update(kw)
    return B.make_adj_params(**base)


def test_adjoint_validation_and_workspace():
    import paper_2411_09605_amd.binding as B
    for kw in [{}, dict(shape_order=1), dict(checkpoint_every=1), dict(checkpoint_every=1000),
               dict(ks=[]), dict(n_steps=1)]:
        assert B.adj_workspace_size(_adj(**kw)) > 0, (kw, B.last_error())
    # checkpoints every step cost more than every 10 steps; one segment of 100 states too
    assert B.adj_workspace_size(_adj(checkpoint_every=1)) > B.adj_workspace_size(_adj())
    assert B.adj_workspace_size(_adj(checkpoint_every=100)) > B.adj_workspace_size(_adj())
    for kw in [dict(n_steps=0), dict(checkpoint_every=0), dict(ks=[0.0]),
               dict(shape_order=3), dict(n_cells=2), dict(dt=-1.0), dict(n_particles=0),
               dict(loss_weight=float("nan"))]:
        assert B.adj_workspace_size(_adj(**kw)) == 0, kw
        assert B.last_error()
    p = _adj()
    p.reserved[1] = 3
    assert B.adj_workspace_size(p) == 0
    p = _adj()
    p.n_modes = 17
    assert B.adj_workspace_size(p) == 0


def test_adjoint_null_handling():
    import paper_2411_09605_amd.binding as B
    assert B.lib.pic_adj_forward(None, None, 0.0, 0.0) == -4
    assert B.lib.pic_adj_backward(None, 1.0) == -4
    assert B.lib.pic_adj_destroy(None) == -4


def test_run_static_rejects_without_a_device():
    """The allocation-free entry point checks its size limit and its buffers before it
    touches a device: an oversized run is PIC_ENOMEM, a caller workspace PIC_EINVAL."""
    import paper_2411_09605_amd.binding as B
    lib = B.lib
    big = _good(n_particles=10_000_000, rebin_every=5)
    assert B.workspace_size(big) > B.STATIC_SCRATCH_BYTES
    buf = B.PicBuffers()
    assert lib.pic_run_static(ctypes.byref(big), ctypes.byref(buf), None, 1, None) == -2
    assert "static workspace" in B.last_error()
    small = _good()
    assert 0 < B.workspace_size(small) <= B.STATIC_SCRATCH_BYTES
    buf.workspace, buf.workspace_bytes = 4096, 1 << 20
    assert lib.pic_run_static(ctypes.byref(small), ctypes.byref(buf), None, 1, None) == -1
    assert "own workspace" in B.last_error()
    assert lib.pic_run_static(ctypes.byref(small), None, None, 1, None) == -1
    assert lib.pic_run_static(ctypes.byref(small), ctypes.byref(B.PicBuffers()), None, -1, None) == -1


def test_deterministic_workspace_holds_partials():
    """The deterministic mode keeps one current replica and a row of partial deposits per
    workgroup (3 N_g doubles each)."""
    import paper_2411_09605_amd as P
    a = _good(n_particles=1_000_000, n_cells=512)
    b = _good(n_particles=1_000_000, n_cells=512, deterministic=True)
    assert P.workspace_size(b) > P.workspace_size(a) + 200 * 3 * 512 * 8


def test_host_input_check_names_the_first_non_finite_value():
    """pic_check_inputs on host arrays (no GPU): finite inputs pass; a NaN or Inf anywhere in
    x, v, w, E or B is PIC_ENONFINITE with its array and index; missing arrays are
    PIC_EINVAL.  Pic.from_arrays runs it before copying anything to the device."""
    import numpy as np
    import paper_2411_09605_amd as P
    import paper_2411_09605_amd.binding as B
    n, ng = 1000, 32
    p = P.make_params(3, "emec_li", 2, n, ng, 10.0, 0.1)
    x, v, w = np.full(n, 0.5), np.zeros((3, n)), np.ones(n)
    E, Bf = np.zeros((3, ng)), np.zeros((2, ng))
    assert B.check_inputs(p, x, v, E, Bf, w) == (0, -1)
    for arr, idx in ((x, 17), (v.reshape(-1), 2 * n + 5), (w, 999), (E.reshape(-1), 64),
                     (Bf.reshape(-1), 33)):
        keep = arr[idx]
        arr[idx] = np.nan if idx % 2 else -np.inf
        rc, bad = B.check_inputs(p, x, v, E, Bf, w)
        assert rc == -5 and bad == idx
        assert "not finite" in P.last_error()
        arr[idx] = keep
    assert B.check_inputs(p, x, v, E, None, w)[0] == -1          # EM needs B
    with pytest.raises(P.PicError) as e:
        P.Pic.check_host_inputs(1, "esec2", 2, ng, 10.0, 0.1, x, np.array([[np.inf] * n]))
    assert e.value.status == -5
