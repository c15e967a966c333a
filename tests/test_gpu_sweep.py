"""The time-step sweep of section 5.1 (Fig. maxerrs_vs_dt) on the GPU against the oracle:
ESEC2, ESEC1 and the standard scheme on small Landau runs in 1D-1V and with two velocity
components, at dt = 0.1, 0.4 and 1.0 over t = 10.  The first 10 steps are compared element
by element (1e-10); over the whole run, where a single particle whose radicand is within
rounding of zero may take the other branch, the fallback totals and energy errors are
compared as statistics, and the paper's claims are checked on the GPU's own records."""
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


def _err(rec):
    t = np.asarray(rec["total"])
    return np.abs(t / t[0] - 1.0).max()


@pytest.mark.parametrize("variant", ["1v", "2v"])
def test_dt_sweep_against_oracle(variant):
    from paper_2411_09605_amd import Pic
    print(f"case: dt sweep {variant}", flush=True)
    builder = workloads.landau if variant == "1v" else workloads.landau_2v
    res = {}
    for dt in (0.1, 0.4, 1.0):
        steps = int(round(10.0 / dt))
        for scheme in ("esec2", "esec1", "standard"):
            wl = builder(n_particles=10_000, n_cells=64, dt=dt, alpha=0.05, steps=steps)
            gu.run_pair(wl, 10, scheme=scheme, every=10)
            g = Pic.from_workload(wl, scheme=scheme, record_capacity=steps + 8)
            g.step(steps)
            gr = g.diagnostics()
            if scheme == "standard":
                o = oracle.StdState(wl)
            else:
                o = oracle.State(wl, scheme)
            o.run(steps)
            orr = np.array(o.records)
            ge, oe = _err(gr), _err(orr)
            gf, of = int(gr["fallbacks"].sum()), int(orr["fallbacks"].sum())
            print(f"  dt {dt} {scheme}: gpu err {ge:.2e} fb {gf}; oracle err {oe:.2e} fb {of}",
                  flush=True)
            assert abs(gf - of) <= 2 + 0.25 * of
            if max(ge, oe) > 1e-13:
                assert ge < 3.0 * oe + 1e-13 and oe < 3.0 * ge + 1e-13
            res[(dt, scheme)] = (ge, gf)
    for dt in (0.1, 0.4, 1.0):
        assert res[(dt, "esec2")][1] <= res[(dt, "esec1")][1]
        assert max(res[(dt, "esec2")][0], 1e-13) <= max(res[(dt, "esec1")][0], 1e-13)
        assert res[(dt, "standard")][0] > 1e3 * max(res[(dt, "esec2")][0], 1e-15) or dt == 1.0
    assert res[(0.1, "esec1")][0] < res[(0.4, "esec1")][0] < res[(1.0, "esec1")][0]
    if variant == "2v":
        assert res[(0.1, "esec2")][0] < 1e-13 and res[(0.4, "esec2")][0] < 1e-13
