"""GPU parity of the batched ensemble form: every run of a batch, advanced together in
persistent launches (and from a replayed hipGraph), against the oracle run alone on the
same seeded inputs, element by element over 10 steps (the 1e-10 bar of tests/gpu_util.py).
"""
import numpy as np
import pytest

import oracle
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


def _run_batch_vs_oracle(runs, steps, every=5, tol=gu.TOL, **knobs):
    from paper_2411_09605_amd import PicBatch
    b = PicBatch(runs, **knobs)
    orcs = [oracle.State(wl) for wl in runs]
    grecs = [[b.diagnostics(k)] for k in range(len(runs))]
    orecs = [[o.run(0)] for o in orcs]
    done = 0
    while done < steps:
        n = min(every, steps - done)
        b.step(n)
        done += n
        for k, (wl, o) in enumerate(zip(runs, orcs)):
            grecs[k].append(b.diagnostics(k))
            orecs[k].append(o.run(n)[1:])
            vscale = max(1.0, float(np.abs(wl.v).max()))
            gu.compare_state(b.state(k), o, wl.length, vscale, wl.scheme == "emec_li", tol,
                             where=f"run {k} step {done}")
    for k in range(len(runs)):
        g, o = np.concatenate(grecs[k]), np.concatenate(orecs[k])
        assert len(g) == steps + 1 and np.array_equal(g["step"], np.arange(steps + 1))
        gu.compare_records(g, o, tol)
    return b


@pytest.mark.parametrize("order", [1, 2])
def test_batched_landau_runs_match_oracle(order):
    """12 Landau runs of uneven size (40 .. 10^4 particles, 32 .. 512 cells)."""
    _say(f"case: batch of 12 landau runs, order {order}")
    runs = workloads.batched_landau(n_runs=12, np_scale=0.01, order=order, steps=10)
    _run_batch_vs_oracle(runs, 10)


@pytest.mark.parametrize("order", [1, 2])
def test_batched_esec1_runs_match_oracle(order):
    """ESEC1 (no predictor current: pass B without its deposit) over 9 Landau runs of uneven
    size."""
    _say(f"case: batch of 9 ESEC1 landau runs, order {order}")
    runs = workloads.batched_landau(n_runs=9, np_scale=0.01, order=order, steps=10)
    for wl in runs:
        wl.scheme = "esec1"
    _run_batch_vs_oracle(runs, 10)


def test_batched_small_launch_shape():
    """Tiny workgroups and chunks with a grid much smaller than the item table, so every
    workgroup strides over items of many runs."""
    _say("case: batch launch shape 64 threads, chunk 128, 5 workgroups")
    runs = workloads.batched_landau(n_runs=7, np_scale=0.005, order=2, steps=10)
    _run_batch_vs_oracle(runs, 10, block_threads=64, chunk=128, grid_blocks=5)


def test_batched_graph_replay_matches_oracle():
    """Steps replayed from a captured 4-step hipGraph (two replays, then 2 plain steps),
    on a stream of its own."""
    import torch
    _say("case: batch hipGraph replay")
    runs = workloads.batched_landau(n_runs=9, np_scale=0.01, order=2, steps=10)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        _run_batch_vs_oracle(runs, 10, every=10, graph_steps=4, stream=s)


def test_batched_graph_replays_repeat():
    """Several calls each replaying the graph, with host synchronisation between them."""
    import torch
    _say("case: batch hipGraph repeated replays")
    runs = workloads.batched_landau(n_runs=5, np_scale=0.01, order=1, steps=12)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        _run_batch_vs_oracle(runs, 12, every=3, graph_steps=3, stream=s)


def test_batched_em_and_es3v():
    """Electromagnetic (EMEC(LI)) runs of different sizes, and electrostatic 1D-3V runs
    with a uniform imposed B and non-uniform weights."""
    _say("case: batch EM weibel x3")
    em = []
    for k, (n, ng) in enumerate([(3000, 64), (20_000, 128), (517, 16)]):
        wl = workloads.weibel(n_particles=n, n_cells=ng, order=2, steps=10, seed=20 + k)
        wl.B0 *= 50.0
        em.append(wl)
    _run_batch_vs_oracle(em, 10)
    _say("case: batch ES 3V x3")
    es = []
    for k, (n, ng) in enumerate([(4001, 40), (900, 12), (12_000, 96)]):
        wl = workloads.landau(n_particles=n, n_cells=ng, alpha=0.1, order=2, seed=30 + k)
        wl.v = np.stack([wl.v[0], workloads.normals(40 + k, 12, n), workloads.normals(40 + k, 14, n)])
        wl.nv = 3
        wl.b_ext = (0.3, -0.6, 1.2)
        wl.w = wl.length / n * (1.0 + 0.5 * workloads.uniforms(40 + k, 20, n))
        es.append(wl)
    _run_batch_vs_oracle(es, 10)


def test_batched_equals_single_run_records():
    """A batch of one run gives the records pic_step gives (same arithmetic)."""
    from paper_2411_09605_amd import Pic, PicBatch
    _say("case: batch of one vs single-run context")
    wl = workloads.two_stream(n_particles=50_000, n_cells=128, steps=8)
    b = PicBatch([wl])
    b.step(8)
    g = Pic.from_workload(wl)
    g.step(8)
    rb, rg = b.diagnostics(0), g.diagnostics()
    for f in ("kinetic", "field_e", "total"):
        assert np.allclose(rb[f], rg[f], rtol=1e-12, atol=0)
    assert np.array_equal(rb["fallbacks"], rg["fallbacks"])


@pytest.mark.timeout(400)
def test_batched_full_ensemble_sampled():
    """The full 512-run ensemble (about 10^8 particles) in the default launch shape:
    5 steps, with 6 runs spread over the size range checked against the oracle."""
    from paper_2411_09605_amd import PicBatch
    _say("case: FULL 512-run batch, sampled runs")
    runs = workloads.batched_landau()
    b = PicBatch(runs)
    b.step(5)
    sizes = np.array([r.n_particles for r in runs])
    pick = list(np.argsort(sizes)[[0, 1, 100, 300, 510, 511]])
    for k in pick:
        wl = runs[k]
        o = oracle.State(wl)
        orec = o.run(5)
        gu.compare_state(b.state(int(k)), o, wl.length, max(1.0, float(np.abs(wl.v).max())),
                         False, where=f"run {k}")
        gu.compare_records(b.diagnostics(int(k)), orec)
    # energy is conserved to roundoff except through Gamma fallbacks (coarse runs with
    # tent shapes and few particles per cell have a few)
    clean = 0
    for k in range(len(runs)):
        if k not in pick:
            rec = b.diagnostics(k)
            assert len(rec) == 6 and rec["nonfinite"].max() == 0, k
            if rec["fallbacks_total"].max() == 0:
                assert rec["rel_energy_err"].max() < 1e-11, k
                clean += 1
    assert clean > 0
