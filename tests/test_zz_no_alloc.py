"""The allocation-free entry point (pic_run_static, static device workspace) against the
context-based one (pic_init + pic_step) on the same inputs: two calls in a row, the second
with a smaller run, each compared element by element to the parity bar (1e-10 relative,
tests/gpu_util.py) together with the newest step's record."""
import numpy as np
import pytest

import workloads
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_09605_amd  # noqa: F401  (raises if the library is missing)


def _static_vs_context(wl, steps):
    import torch
    import paper_2411_09605_amd as P
    ref = P.Pic.from_workload(wl, device="cuda:0")
    ref.step(steps)
    rrec = ref.diagnostics()
    rst = ref.state()
    # the same inputs as fresh device arrays for the static call
    f64 = dict(dtype=torch.float64, device="cuda:0")
    n = wl.n_particles
    x = torch.as_tensor(np.ascontiguousarray(wl.x, dtype=np.float64)).to(**f64)
    v = torch.as_tensor(np.ascontiguousarray(wl.v, dtype=np.float64).reshape(wl.nv, n)).to(**f64)
    E = torch.zeros((3, wl.n_cells), **f64)
    if wl.E0 is not None:
        E.copy_(torch.as_tensor(np.asarray(wl.E0, dtype=np.float64).reshape(3, -1)))
    B = None
    if wl.scheme == "emec_li":
        B = torch.zeros((2, wl.n_cells), **f64)
        if wl.B0 is not None:
            B.copy_(torch.as_tensor(np.asarray(wl.B0, dtype=np.float64).reshape(2, -1)))
    params = P.make_params(wl.nv, wl.scheme, wl.order, n, wl.n_cells, wl.length, wl.dt,
                           c=wl.c, b_ext=wl.b_ext, init_gauss=wl.init_gauss)
    assert P.workspace_size(params) <= P.STATIC_SCRATCH_BYTES
    diag = torch.zeros(P.DIAG_DTYPE.itemsize, dtype=torch.uint8, device="cuda:0")
    P.run_static(params, x, v, E, B=B, n_steps=steps, diag=diag)
    torch.cuda.synchronize()
    rec = P.diag_from_tensor(diag)
    L = wl.length
    assert gu.periodic_err(x.cpu().numpy(), rst["x"], L).max() <= gu.TOL * L
    vs = max(1.0, float(np.abs(wl.v).max()))
    assert np.abs(v.cpu().numpy() - rst["v"]).max() <= gu.TOL * vs
    Eh = E.cpu().numpy()
    for c in range(3 if wl.scheme == "emec_li" else 1):
        sc = max(np.abs(rst["E"][c]).max(), 1e-300)
        assert np.abs(Eh[c] - rst["E"][c]).max() <= gu.TOL * sc
    if B is not None:
        Bh = B.cpu().numpy()
        for c in range(2):
            sc = max(np.abs(rst["B"][c]).max(), 1e-300)
            assert np.abs(Bh[c] - rst["B"][c]).max() <= gu.TOL * sc
    last = rrec[-1]
    assert rec["step"] == last["step"] == steps
    te0 = rrec["total"][0]
    for f in ("kinetic", "field_e", "field_b", "total"):
        assert abs(rec[f] - last[f]) <= gu.TOL * te0, f
    assert rec["fallbacks_total"] == last["fallbacks_total"]
    ref.destroy()


def test_static_entry_point_two_calls():
    """A two-stream run, then a smaller electromagnetic one in the same process: the
    second call reuses the static workspace the first one left behind."""
    print("case: pic_run_static two-stream 2e5 x 512, 10 steps", flush=True)
    _static_vs_context(workloads.two_stream(n_particles=200_000, n_cells=512, steps=10), 10)
    print("case: pic_run_static weibel 3e4 x 64, 6 steps", flush=True)
    wl = workloads.weibel(n_particles=30_000, n_cells=64, steps=6)
    wl.B0 *= 50.0
    _static_vs_context(wl, 6)
