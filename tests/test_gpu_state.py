"""GPU tests of the deterministic mode and of checkpoint/resume (pic_save_state /
pic_load_state), through the C ABI.

* Deterministic mode: two runs give bit-identical states and records; it agrees with
  the default mode to 1e-12 (the metric of tests/gpu_util.py) over 10 steps and with the
  oracle to the parity bar.
* Resume: a state saved at step 10 and loaded into a fresh context continues to step 20
  bit for bit like the uninterrupted run (deterministic mode), or to the parity bar
  (default mode, where the order of the FP64 current sums varies).
* The fixed-point deposit against the FP64-atomic one at the Weibel workload's size.
"""
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
    import paper_2411_09605_amd  # noqa: F401


def _say(msg):
    print(msg, flush=True)


def _bitwise_equal(a, b):
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def _records_equal(ra, rb):
    for f in ("step", "kinetic", "field_e", "field_b", "total", "max_gamma_dev",
              "fallbacks", "fallbacks_total", "nonfinite"):
        assert np.array_equal(ra[f], rb[f]), f


def _cases():
    ts = workloads.two_stream(n_particles=300_001, n_cells=256, steps=20)
    em = workloads.weibel(n_particles=100_000, n_cells=128, steps=20)
    em.B0 *= 50.0
    lf = workloads.weibel(n_particles=100_000, n_cells=128, steps=20, dt=0.08)
    lf.B0 *= 50.0
    return [("two-stream 3e5 x 256", ts, {}), ("weibel 1e5 x 128", em, {}),
            ("two-stream interleaved", ts, dict(interleave=True)),
            ("two-stream esec1 (one pass)", ts, dict(scheme="esec1")),
            ("weibel 1e5 x 128 emec_psatd", em, dict(scheme="emec_psatd")),
            ("weibel 1e5 x 128 emec_lf", lf, dict(scheme="emec_lf"))]


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4, 5])
def test_deterministic_runs_are_bit_identical(k):
    from paper_2411_09605_amd import Pic
    name, wl, kn = _cases()[k]
    _say(f"case: deterministic reruns, {name}")
    runs = []
    for _ in range(2):
        g = Pic.from_workload(wl, deterministic=True, **kn)
        g.step(15)
        runs.append((g.state(), g.diagnostics()))
        g.destroy()
    _bitwise_equal(runs[0][0], runs[1][0])
    _records_equal(runs[0][1], runs[1][1])


@pytest.mark.parametrize("k", [0, 1])
def test_deterministic_matches_default_and_oracle(k):
    """10 steps: deterministic vs default to 1e-12, deterministic vs the oracle to the
    parity bar (with its records)."""
    from paper_2411_09605_amd import Pic
    name, wl, _ = _cases()[k]
    _say(f"case: deterministic vs default vs oracle, {name}")
    grec, orec, gdet, ost = gu.run_pair(wl, 10, every=5, deterministic=True)
    ref = Pic.from_workload(wl)
    ref.step(10)
    em = wl.scheme == "emec_li"
    st = ref.state()
    vscale = max(1.0, float(np.abs(wl.v).max()))

    class _O:                                  # the default run in the oracle's shape
        x, v, E = st["x"], st["v"], st["E"]
        B = st.get("B")
    gu.compare_state(gdet.state(), _O, wl.length, vscale, em, tol=1e-12, where="det vs default")


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4, 5])
def test_resume_is_bit_identical_in_deterministic_mode(k):
    from paper_2411_09605_amd import Pic
    name, wl, kn = _cases()[k]
    _say(f"case: save at 10, resume to 20, deterministic, {name}")
    a = Pic.from_workload(wl, deterministic=True, **kn)
    a.step(20)
    sa, ra = a.state(), a.diagnostics()
    b = Pic.from_workload(wl, deterministic=True, **kn)
    b.step(10)
    blob = b.save_state()
    b.step(3)                                   # the saver moves on; the blob stays
    c = Pic.from_workload(wl, deterministic=True, **kn)
    c.step(2)                                   # whatever the loader did before
    c.diagnostics()
    c.load_state(blob)
    c.step(10)
    sc, rc = c.state(), c.diagnostics()
    _bitwise_equal(sa, sc)
    assert rc["step"][0] == 10 and rc["step"][-1] == 20
    _records_equal(ra[10:], rc)


def test_resume_default_mode_and_rebin_with_ids_and_weights():
    """Default mode: the resumed run matches the uninterrupted one to the parity bar,
    also with rebins every 3 steps, tracked ids and non-uniform weights (the library's
    permuted copy of the weights is part of the state)."""
    from paper_2411_09605_amd import Pic
    _say("case: resume, default mode (plain and rebin + ids + weights)")
    n = 40_001
    wl = workloads.landau(n_particles=n, n_cells=40, alpha=0.1, order=2)
    wl.v = np.stack([wl.v[0], workloads.normals(9, 12, n), workloads.normals(9, 14, n)])
    wl.nv = 3
    wl.b_ext = (0.3, -0.6, 1.2)
    wl.w = wl.length / n * (1.0 + 0.5 * workloads.uniforms(9, 20, n))
    for kn in ({}, dict(rebin_every=3, track_ids=True)):
        a = Pic.from_workload(wl, **kn)
        a.step(20)
        sa = gu.order_by_ids(a.state())
        ra = a.diagnostics()
        b = Pic.from_workload(wl, **kn)
        b.step(10)
        blob = b.save_state()
        c = Pic.from_workload(wl, **kn)
        c.load_state(blob)
        c.step(10)
        sc = gu.order_by_ids(c.state())
        rc = c.diagnostics()
        assert gu.periodic_err(sc["x"], sa["x"], wl.length).max() <= gu.TOL * wl.length
        assert np.abs(sc["v"] - sa["v"]).max() <= gu.TOL * np.abs(wl.v).max()
        assert np.abs(sc["E"] - sa["E"]).max() <= gu.TOL * np.abs(sa["E"]).max()
        te0 = ra["total"][0]
        assert np.abs(rc["total"] - ra["total"][10:]).max() <= gu.TOL * te0
        assert np.array_equal(rc["fallbacks_total"], ra["fallbacks_total"][10:])


def test_load_rejects_other_runs_and_leaves_state():
    from paper_2411_09605_amd import Pic, PicError
    _say("case: load_state rejects mismatches")
    wl = workloads.two_stream(n_particles=20_000, n_cells=64, steps=5)
    a = Pic.from_workload(wl)
    a.step(3)
    blob = a.save_state()
    other = workloads.two_stream(n_particles=20_000, n_cells=128, steps=5)
    for bad_ctx, bad_blob in [(Pic.from_workload(other), blob),
                              (Pic.from_workload(wl, deterministic=True), blob),
                              (Pic.from_workload(wl), blob[:100]),
                              (Pic.from_workload(wl), np.zeros_like(blob))]:
        before = bad_ctx.state()
        with pytest.raises(PicError) as e:
            bad_ctx.load_state(bad_blob)
        assert e.value.status == -1
        _bitwise_equal(before, bad_ctx.state())
        bad_ctx.destroy()


@pytest.mark.timeout(900)
def test_weibel_full_size_fixed_point_vs_fp64_deposit():
    """At the Weibel workload's size (2e7 particles, 256 cells, interleaved batches) the
    fixed-point LDS deposit (scale from the run's fastest particle) and FP64 LDS atomics
    agree to 1e-12 over 10 steps."""
    from paper_2411_09605_amd import Pic
    _say("case: weibel FULL, fixed-point vs FP64 LDS deposit, 10 steps")
    wl = workloads.weibel()
    a = Pic.from_workload(wl)
    b = Pic.from_workload(wl, deposit_mode="lds_f64")
    a.step(10)
    b.step(10)
    sa, sb = a.state(), b.state()

    class _O:
        x, v, E, B = sb["x"], sb["v"], sb["E"], sb["B"]
    gu.compare_state(sa, _O, wl.length, float(np.abs(wl.v).max()), True, tol=1e-12,
                     where="fixed point vs FP64")
