"""Pins of the oracle's standard explicit PIC scheme (the comparison scheme of section 5:
Vlasov-Poisson with the symmetric leapfrog/Boris push, eq. (symm_Boris)), against what the
paper and the mathematics fix, independently of the oracle's own code:

* with zero weights there is no charge, so no field: the push is the symmetric Boris
  rotation in the imposed B (an independent 3x3 solve) and free streaming without B;
* total momentum sum_p w_p v_p is conserved exactly (deposit and gather share the shape
  and the spectral Gauss solve's kernel is odd, so the self-force cancels);
* the binomial filter's closed form: mode m is scaled by cos^2(pi m / N);
* second-order self-convergence in dt;
* Landau damping and two-stream growth at the kinetic rates;
* energy is not conserved: its error is many orders of magnitude above ESEC2's on the
  same run (section 5.2), and shrinks like dt^2.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from tests import theory
from tests.test_oracle_pins import _boris_reference, _landau_3v


def _energy_err(recs):
    t = np.array(recs)["total"]
    return np.abs(t / t[0] - 1.0).max()


def test_zero_weight_is_boris_and_free_streaming():
    n, steps, dt = 64, 25, 0.3
    wl = _landau_3v(n=n, b_ext=(0.4, -1.3, 2.0))
    wl.w = np.zeros(n)
    wl.dt = dt
    st = oracle.StdState(wl)
    x0, v0 = np.mod(st.x, wl.length), st.v.copy()
    st.run(steps)
    xr, vr = _boris_reference(x0, v0, wl.b_ext, dt, wl.length, steps)
    dx = np.abs(st.x - xr)
    assert np.max(np.minimum(dx, wl.length - dx)) < 1e-12
    assert np.max(np.abs(st.v - vr)) < 1e-12
    assert np.abs(st.E).max() == 0.0
    # 1D-1V: free streaming
    w1 = workloads.landau(n_particles=100, n_cells=16, order=2)
    w1.w = np.zeros(100)
    s1 = oracle.StdState(w1)
    s1.run(10)
    xe = np.mod(np.mod(w1.x, w1.length) + 10 * w1.dt * w1.v[0], w1.length)
    d = np.abs(s1.x - xe)
    assert np.max(np.minimum(d, w1.length - d)) < 1e-12
    assert np.array_equal(s1.v, w1.v)


@pytest.mark.parametrize("order,filt", [(1, False), (2, False), (2, True)])
def test_momentum_is_conserved(order, filt):
    wl = workloads.two_stream(n_particles=20_000, n_cells=64, alpha=0.05, order=order)
    w = wl.length / wl.n_particles
    p0 = w * wl.v[0].sum()
    scale = w * np.abs(wl.v[0]).sum()
    st = oracle.StdState(wl, filter_rho=filt)
    st.run(60)
    assert abs(w * st.v[0].sum() - p0) < 1e-13 * scale


def test_binomial_filter_closed_form():
    N = 32
    i = np.arange(N)
    for m in (0, 1, 5, 15, 16):
        f = np.cos(2 * np.pi * m * i / N)
        g = oracle.binomial(f)
        assert np.allclose(g, math.cos(math.pi * m / N) ** 2 * f, rtol=0, atol=1e-14)
    rng = np.random.default_rng(1)
    f = rng.normal(size=N)
    assert abs(oracle.binomial(f).sum() - f.sum()) < 1e-13
    assert np.abs(oracle.binomial(np.cos(np.pi * i))).max() < 1e-15      # Nyquist removed


def test_second_order_self_convergence():
    res = []
    L = None
    for dt in (0.1, 0.05, 0.025, 0.0125):
        wl = workloads.landau(n_particles=4000, n_cells=16, alpha=0.3, quiet=True, order=2,
                              dt=dt)
        L = wl.length
        st = oracle.StdState(wl)
        st.run(int(round(2.0 / dt)))
        res.append((st.x.copy(), st.v[0].copy()))

    def err(a, b):
        d = np.abs(a[0] - b[0])
        d = np.minimum(d, L - d)
        return math.sqrt(np.mean(d ** 2) + np.mean((a[1] - b[1]) ** 2))
    e = [err(res[i], res[i + 1]) for i in range(3)]
    ratios = np.array(e[:-1]) / np.array(e[1:])
    assert np.all((ratios > 3.6) & (ratios < 4.5)), ratios


def test_landau_damping_rate():
    wl = workloads.landau(quiet=True, steps=130)
    st = oracle.StdState(wl)
    st.run(0)
    amp = [theory.mode_amplitude(st.E[0], 1)]
    for _ in range(wl.steps):
        st.run(1)
        amp.append(theory.mode_amplitude(st.E[0], 1))
    amp = np.array(amp)
    # the fields are at half steps: E^{n-1/2} after step n
    t = np.concatenate([[0.0], (np.arange(wl.steps) + 0.5) * wl.dt])
    pk = [i for i in range(1, len(amp) - 1) if amp[i] > amp[i - 1] and amp[i] >= amp[i + 1]]
    pk = [i for i in pk if 2.0 <= t[i] <= 12.5]
    gamma = np.polyfit(t[pk], np.log(amp[pk]), 1)[0]
    ref = theory.landau_root(0.5).imag
    assert abs(gamma - ref) < 0.03 * abs(ref), (gamma, ref)


def test_two_stream_growth_rate_and_energy_against_esec2():
    wl = workloads.two_stream(n_particles=100_000, n_cells=128, alpha=1e-4, quiet=True,
                              steps=400)
    st = oracle.StdState(wl)
    st.run(0)
    amp = []
    for _ in range(wl.steps):
        st.run(1)
        amp.append(theory.mode_amplitude(st.E[0], 1))
    t = (np.arange(wl.steps) + 0.5) * wl.dt
    sel = (t > 12) & (t < 20)
    gamma = np.polyfit(t[sel], np.log(np.array(amp)[sel]), 1)[0]
    ref = theory.two_stream_warm_growth(0.2, 3.0, 0.1)
    assert abs(gamma - ref) < 0.02 * ref, (gamma, ref)
    # section 5.2: ESEC2 conserves energy many orders of magnitude better
    es = oracle.State(wl)
    es.run(wl.steps)
    e_std, e_es2 = _energy_err(st.records), _energy_err(es.records)
    assert e_std > 1e5 * max(e_es2, 1e-16), (e_std, e_es2)


def test_energy_error_shrinks_like_dt_squared():
    errs = []
    for dt in (0.2, 0.1, 0.05):
        wl = workloads.landau(n_particles=20_000, n_cells=32, alpha=0.2, quiet=True,
                              order=2, dt=dt)
        st = oracle.StdState(wl)
        st.run(int(round(4.0 / dt)))
        errs.append(_energy_err(st.records))
    r = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all((r > 3.0) & (r < 5.0)), (errs, r)
