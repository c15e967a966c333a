"""Pins of the whole oracle step against what the paper and the mathematics fix (no GPU).

* total energy (section 5.1) is conserved exactly in exact arithmetic when no fallback
  occurs (eq. (exp_econs_simple); eq. (still_e_dot_j) with (EM_econs) for EMEC(LI)):
  here to ~1e-13 relative in FP64;
* with E = 0 and w = 0 the particle push is the symmetric Boris scheme
  (eq. (symm_Boris), section 3.2 end), checked against an independent 3x3 linear solve;
  with E = B = 0 it is free streaming;
* Gamma - 1 = O(dt^3) for ESEC1 (section 3.2) and O(dt^4) for ESEC2 (section 3.3,
  Appendix A): one-step halving ratios tend to 8 and 16;
* the scheme is second order (section 3.2): self-convergence ratio 4 per halving;
* in 1D electrostatics E = -grad(phi) has zero mean, kept by the Ampere update;
* physics: linear Landau damping (section 5.1) and two-stream growth (section 5.2) match
  the kinetic dispersion roots; Weibel growth (section 5.3) is in the right range;
* ESEC2 has fewer imaginary-Gamma particles than ESEC1 (section 5.1).
"""
import copy
import math

import numpy as np
import pytest

import oracle
import workloads
from tests import theory


def _rel_energy_drift(rec):
    te = rec["total"]
    return np.max(np.abs(te - te[0])) / te[0]


def _landau_3v(n=20000, b_ext=(0.3, -0.5, 1.1), order=2, steps=60):
    wl = workloads.landau(n_particles=n, n_cells=32, alpha=0.1, order=order, steps=steps)
    vy = workloads.normals(7, 12, n)
    vz = workloads.normals(7, 14, n)
    wl.v = np.stack([wl.v[0], vy, vz])
    wl.nv = 3
    wl.b_ext = b_ext
    return wl


def test_energy_landau_full():
    """The Landau workload (64 cells, 1e5 particles, tent, dt 0.1, 200 steps)."""
    wl = workloads.landau()
    rec = oracle.State(wl).run(wl.steps)
    assert _rel_energy_drift(rec) < 1e-13
    assert rec["nonfinite"].max() == 0


def test_energy_two_stream_quadratic():
    wl = workloads.two_stream(n_particles=50_000, n_cells=512, steps=100)
    rec = oracle.State(wl).run(wl.steps)
    assert _rel_energy_drift(rec) < 1e-12


def test_energy_es_3v_external_field():
    wl = _landau_3v()
    rec = oracle.State(wl).run(wl.steps)
    assert rec["fallbacks"].sum() == 0
    assert _rel_energy_drift(rec) < 1e-13


def test_energy_em_li():
    wl = workloads.weibel(n_particles=20_000, n_cells=64, steps=60)
    wl.B0[1] *= 30.0          # larger seed so that field energy matters
    rec = oracle.State(wl).run(wl.steps)
    assert rec["field_b"][0] > 0
    assert _rel_energy_drift(rec) < 1e-13


def _boris_reference(x, v, b, dt, L, steps):
    """Symmetric Boris (eq. symm_Boris) with E = 0: x* = x + dt/2 v;
    (I - dt/2 [.xB]) v' = (I + dt/2 [.xB]) v;  x' = x* + dt/2 v'."""
    M = np.array([[0, b[2], -b[1]], [-b[2], 0, b[0]], [b[1], -b[0], 0]])  # M a = a x b
    A = np.eye(3) - 0.5 * dt * M
    Bm = np.eye(3) + 0.5 * dt * M
    x = x.copy()
    v = v.copy()
    for _ in range(steps):
        xs = x + 0.5 * dt * v[0]
        v = np.linalg.solve(A, Bm @ v)
        x = xs + 0.5 * dt * v[0]
    return np.mod(x, L), v


@pytest.mark.parametrize("scheme", ["esec2", "esec1", "emec_li"])
def test_boris_special_case(scheme):
    n, steps, dt = 64, 25, 0.3
    wl = _landau_3v(n=n, b_ext=(0.4, -1.3, 2.0))
    wl.w = np.zeros(n)                  # no current, so E stays zero
    wl.scheme, wl.dt = scheme, dt
    wl.init_gauss = False
    wl.E0 = np.zeros((3, wl.n_cells))
    wl.B0 = np.zeros((2, wl.n_cells))
    st = oracle.State(wl)
    x0, v0 = st.x.copy(), st.v.copy()
    rec = st.run(steps)
    xr, vr = _boris_reference(x0, v0, wl.b_ext, dt, wl.length, steps)
    dx = np.abs(st.x - xr)
    assert np.max(np.minimum(dx, wl.length - dx)) < 1e-12
    assert np.max(np.abs(st.v - vr)) < 1e-12
    # the magnetic field does no work
    assert np.max(np.abs(np.sum(st.v ** 2, 0) - np.sum(v0 ** 2, 0))) < 1e-12
    assert rec["fallbacks"].sum() == 0 and rec["max_gamma_dev"].max() < 1e-14


def test_free_streaming():
    wl = workloads.landau(n_particles=500, n_cells=16, steps=7)
    wl.w = np.zeros(500)
    wl.init_gauss = False
    st = oracle.State(wl)
    x0, v0 = st.x.copy(), st.v.copy()
    rec = st.run(7)
    assert np.array_equal(st.v, v0)
    d = np.abs(st.x - np.mod(x0 + 7 * wl.dt * v0[0], wl.length))
    assert np.max(np.minimum(d, wl.length - d)) < 1e-12
    assert rec["max_gamma_dev"].max() == 0.0


def test_field_mean_stays_zero():
    wl = workloads.landau(n_particles=20_000, n_cells=32, steps=50)
    wl.v = wl.v + 0.7                   # net drift: the raw current has a large mean
    st = oracle.State(wl)
    for _ in range(5):
        st.run(10)
        assert abs(st.E[0].sum()) < 1e-13 * max(1.0, np.abs(st.E[0]).max()) * wl.n_cells


def _gamma_spread(scheme, order):
    wl = workloads.landau(n_particles=20_000, n_cells=32, alpha=0.3, quiet=True,
                          order=order, dt=0.025)
    base = oracle.State(wl, scheme=scheme)
    base.run(40)                        # t = 1: large current, so dE/dt != 0
    med = []
    for dt in (0.1, 0.05, 0.025):
        st = copy.deepcopy(base)
        st.cfg = oracle.make_cfg(1, scheme, order, wl.n_cells, wl.n_particles, wl.length, dt)
        g = np.zeros(wl.n_particles)
        v0 = st.v[0].copy()
        st.run(1, gamma_out=g)
        med.append(np.median(np.abs(g[np.abs(v0) > 0.5] - 1.0)))
    return np.array(med)


@pytest.mark.parametrize("order", [1, 2])
def test_gamma_order_esec1_vs_esec2(order):
    m1 = _gamma_spread("esec1", order)
    m2 = _gamma_spread("esec2", order)
    r1 = m1[:-1] / m1[1:]
    r2 = m2[:-1] / m2[1:]
    assert 7.0 < r1[-1] < 9.0            # Gamma - 1 = O(dt^3)
    assert 14.0 < r2[-1] < 18.0          # Gamma - 1 = O(dt^4)
    assert np.all(m2 < m1)


def test_second_order_convergence():
    L = None
    res = []
    for dt in (0.1, 0.05, 0.025, 0.0125):
        wl = workloads.landau(n_particles=4000, n_cells=16, alpha=0.3, quiet=True, order=2,
                              dt=dt)
        L = wl.length
        st = oracle.State(wl)
        st.run(int(round(2.0 / dt)))
        res.append((st.x.copy(), st.v[0].copy()))

    def err(a, b):
        d = np.abs(a[0] - b[0])
        d = np.minimum(d, L - d)
        return math.sqrt(np.mean(d ** 2) + np.mean((a[1] - b[1]) ** 2))
    e = [err(res[i], res[i + 1]) for i in range(3)]
    ratios = np.array(e[:-1]) / np.array(e[1:])
    assert np.all((ratios > 3.6) & (ratios < 4.5)), ratios


def test_fallbacks_esec2_fewer_than_esec1():
    wl = workloads.landau(steps=100)
    r2 = oracle.State(wl, "esec2").run(100)
    r1 = oracle.State(wl, "esec1").run(100)
    assert r2["fallbacks"].sum() < r1["fallbacks"].sum()
    assert _rel_energy_drift(r2) < _rel_energy_drift(r1)


def test_landau_damping_rate():
    k = 0.5
    wl = workloads.landau(quiet=True, steps=130)
    st = oracle.State(wl)
    amp = [theory.mode_amplitude(st.E[0], 1)]
    for _ in range(wl.steps):
        st.run(1)
        amp.append(theory.mode_amplitude(st.E[0], 1))
    amp = np.array(amp)
    t = np.arange(len(amp)) * wl.dt
    pk = [i for i in range(1, len(amp) - 1) if amp[i] > amp[i - 1] and amp[i] >= amp[i + 1]]
    pk = [i for i in pk if 2.0 <= t[i] <= 12.5]
    gamma = np.polyfit(t[pk], np.log(amp[pk]), 1)[0]
    w = theory.landau_root(k)
    assert abs(gamma - w.imag) < 0.03 * abs(w.imag), (gamma, w)
    # successive |E_1| maxima are half a period apart
    omega = math.pi / np.mean(np.diff(t[pk]))
    assert abs(omega - w.real) < 0.03 * w.real
    # the approximate rate printed in section 5.1 is only rough at k = 0.5
    approx, bohm_gross = theory.landau_rate_paper_approx(k)
    assert 1.0 < approx / abs(w.imag) < 2.0 and abs(bohm_gross - w.real) < 0.1


def test_two_stream_growth_rate():
    wl = workloads.two_stream(n_particles=100_000, n_cells=128, alpha=1e-4, quiet=True,
                              steps=400)
    st = oracle.State(wl)
    amp = []
    for _ in range(wl.steps):
        st.run(1)
        amp.append(theory.mode_amplitude(st.E[0], 1))
    t = (np.arange(wl.steps) + 1) * wl.dt
    sel = (t > 12) & (t < 20)
    gamma = np.polyfit(t[sel], np.log(np.array(amp)[sel]), 1)[0]
    ref = theory.two_stream_warm_growth(0.2, 3.0, 0.1)
    assert abs(gamma - ref) < 0.02 * ref, (gamma, ref)
    assert _rel_energy_drift(np.array(st.records)) < 1e-12


def test_weibel_growth_in_range():
    wl = workloads.weibel(n_particles=20_000, n_cells=32, dt=0.1, steps=400)
    st = oracle.State(wl)
    amp = []
    for _ in range(wl.steps):
        st.run(1)
        amp.append(theory.mode_amplitude(st.B[1], 1))
    amp = np.array(amp)
    t = (np.arange(wl.steps) + 1) * wl.dt
    sel = (t > 8) & (t < 35)
    gamma = np.polyfit(t[sel], np.log(amp[sel]), 1)[0]
    ref = theory.weibel_growth(0.5, 0.15, 0.3)
    assert 0.65 * ref < gamma < 1.1 * ref, (gamma, ref)
    assert amp[-1] > 5 * amp[0]
    assert _rel_energy_drift(np.array(st.records)) < 1e-12


@pytest.mark.slow
def test_weibel_growth_rate_quiet_positions():
    """Weibel growth (section 5.3) with 2e5 particles on 64 cells, quiet-start positions and
    dt = 0.1: the seeded mode grows at the bi-Maxwellian kinetic rate (0.0827 at k = 0.5)
    within 5% over the linear phase t in (15, 40); energy holds to 1e-12."""
    wl = workloads.weibel(n_particles=200_000, n_cells=64, dt=0.1, steps=450)
    st = oracle.State(wl)
    amp = []
    for _ in range(wl.steps):
        st.run(1)
        amp.append(theory.mode_amplitude(st.B[1], 1))
    amp = np.array(amp)
    t = (np.arange(wl.steps) + 1) * wl.dt
    sel = (t > 15) & (t < 40)
    gamma = np.polyfit(t[sel], np.log(amp[sel]), 1)[0]
    ref = theory.weibel_growth(0.5, 0.15, 0.3)
    assert abs(gamma - ref) < 0.05 * ref, (gamma, ref)
    # the linear phase is a straight line in log |B_1|: the fit's residuals are small
    res = np.log(amp[sel]) - np.polyval(np.polyfit(t[sel], np.log(amp[sel]), 1), t[sel])
    assert np.abs(res).max() < 0.1
    assert _rel_energy_drift(np.array(st.records)) < 1e-12


def test_dt_sweep_fallbacks_and_energy_section_5_1():
    """Section 5.1 (Fig. maxerrs_vs_dt): with the paper's two velocity components, ESEC2
    keeps energy to rounding up to dt = 0.7 with no fallback, while ESEC1's fallbacks and
    energy error grow with dt; in 1D-1V (where |v-dagger| near zero is far more likely)
    ESEC2 still has fewer fallbacks and a smaller error than ESEC1 at every dt."""
    e1, f1 = [], []
    for dt in (0.1, 0.4, 0.7):
        steps = int(round(10.0 / dt))
        for wlf in (workloads.landau_2v, workloads.landau):
            r2 = oracle.State(wlf(n_particles=10_000, dt=dt, alpha=0.05), "esec2").run(steps)
            r1 = oracle.State(wlf(n_particles=10_000, dt=dt, alpha=0.05), "esec1").run(steps)
            assert r2["fallbacks"].sum() <= r1["fallbacks"].sum()
            # (below 1e-13 both are rounding)
            assert max(_rel_energy_drift(r2), 1e-13) <= max(_rel_energy_drift(r1), 1e-13)
            if wlf is workloads.landau_2v:
                assert r2["fallbacks"].sum() == 0 and _rel_energy_drift(r2) < 1e-13, dt
                e1.append(_rel_energy_drift(r1))
                f1.append(r1["fallbacks"].sum())
    assert e1[0] < e1[1] < e1[2] and f1[0] <= f1[1] <= f1[2] and f1[2] > f1[0]
