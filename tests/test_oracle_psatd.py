"""Pins of the oracle's EMEC(PSATD) (section 4.2, eq. (EM_PSATD); field solve eq.
(PSATDformula) and its time average), against what the mathematics fixes independently of
the oracle's own code:

* vacuum: a single travelling light wave on the staggered grid advances by exactly
  omega dt = c k dt per step (no dispersion error, unlike Crank-Nicolson), for both
  polarisations, and the step's time average equals the analytic integral;
* a driven mode: the solve with a fixed current matches a fine Runge-Kutta integration of
  the same semi-discrete system, whose staggered spectral curls are built here with numpy's
  FFT;
* energy: with particles, total energy (section 5.1) is conserved to rounding (eq.
  (PSATDecons) with the particle identity);
* the Boris limit (zero weights, uniform imposed B) and the Weibel growth rate.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from tests import theory
from tests.test_oracle_pins import _boris_reference, _landau_3v


def _grid(ng, L):
    h = L / ng
    return h, np.arange(ng) * h, (np.arange(ng) + 0.5) * h


@pytest.mark.parametrize("m", [1, 3, 15])
def test_vacuum_wave_is_exact_and_average(m):
    ng, L, c, dt = 32, 4 * math.pi, 1.3, 0.3
    h, xn, xh = _grid(ng, L)
    k = 2 * math.pi * m / L
    w = c * k
    J = np.zeros((3, ng))
    for pol in (0, 1):
        E = np.zeros((3, ng))
        B = np.zeros((2, ng))
        if pol == 0:              # E_y = c B_z travels towards +x
            E[1], B[1] = np.cos(k * xn), np.cos(k * xh) / c
        else:                     # E_z = -c B_y travels towards +x
            E[2], B[0] = np.cos(k * xn), -np.cos(k * xh) / c
        Eo, Bo, Ea = oracle.psatd(ng, L, c, dt, E, B, J)
        ec = 1 + pol
        assert np.abs(Eo[ec] - np.cos(k * xn - w * dt)).max() < 1e-13
        bc, sgn = (1, 1.0) if pol == 0 else (0, -1.0)
        assert np.abs(Bo[bc] - sgn * np.cos(k * xh - w * dt) / c).max() < 1e-13
        avg = (np.sin(k * xn) - np.sin(k * xn - w * dt)) / (w * dt)
        assert np.abs(Ea[ec] - avg).max() < 1e-13
        assert np.abs(Eo[0]).max() == 0 and np.abs(Eo[3 - ec]).max() == 0


def test_vacuum_many_steps_no_dispersion_against_crank_nicolson():
    """100 steps of a short wave (8 cells per wavelength): PSATD keeps the exact phase; the
    run through the oracle's EMEC(LI) field solve (Crank-Nicolson with centred differences)
    lags measurably."""
    ng, L, c, dt, steps = 64, 4 * math.pi, 1.0, 0.2, 100
    h, xn, xh = _grid(ng, L)
    k = 2 * math.pi * 8 / L
    wl = _landau_3v(n=4, b_ext=(0.0, 0.0, 0.0))
    wl.n_cells, wl.length, wl.dt, wl.c = ng, L, dt, c
    wl.x = np.linspace(0.1, L - 0.1, 4)
    wl.w = np.zeros(4)
    wl.init_gauss = False
    wl.E0 = np.zeros((3, ng))
    wl.B0 = np.zeros((2, ng))
    wl.E0[1], wl.B0[1] = np.cos(k * xn), np.cos(k * xh) / c
    res = {}
    for sch in ("emec_psatd", "emec_li"):
        st = oracle.State(wl, sch)
        st.run(steps)
        res[sch] = np.abs(st.E[1] - np.cos(k * xn - c * k * dt * steps)).max()
    assert res["emec_psatd"] < 1e-12
    assert res["emec_li"] > 1e-2


def _stag_rhs(E, B, J, c, L):
    """Semi-discrete Maxwell on the staggered grid with spectral curls (numpy FFT):
    dE/dt = c^2 curl B - j, dB/dt = -curl E, E, j on nodes, B on half nodes."""
    ng = E.shape[1]
    h = L / ng
    m = np.fft.fftfreq(ng, 1.0 / ng)
    k = 2 * np.pi * m / L
    a = 1j * k * np.exp(0.5j * k * h)      # d/dx from nodes to half nodes
    b = 1j * k * np.exp(-0.5j * k * h)     # d/dx from half nodes to nodes
    if ng % 2 == 0:                        # the Nyquist mode: both symbols are real
        a[ng // 2], b[ng // 2] = -np.pi / h, np.pi / h
    dp = lambda f: np.real(np.fft.ifft(a * np.fft.fft(f)))   # noqa: E731
    dm = lambda g: np.real(np.fft.ifft(b * np.fft.fft(g)))   # noqa: E731
    dE = np.zeros_like(E)
    dB = np.zeros_like(B)
    dE[0] = -J[0]
    dE[1] = -c * c * dm(B[1]) - J[1]      # (curl B)_y = -d B_z/dx
    dE[2] = c * c * dm(B[0]) - J[2]       # (curl B)_z = +d B_y/dx
    dB[0] = dp(E[2])                      # -(curl E)_y = +d E_z/dx
    dB[1] = -dp(E[1])                     # -(curl E)_z = -d E_y/dx
    return dE, dB


def test_driven_modes_match_fine_runge_kutta():
    rng = np.random.default_rng(4)
    ng, L, c, tau = 16, 5.0, 0.8, 0.37
    E = rng.normal(size=(3, ng))
    B = rng.normal(size=(2, ng))
    J = rng.normal(size=(3, ng))
    Eo, Bo, Ea = oracle.psatd(ng, L, c, tau, E, B, J)
    n = 4000
    dt = tau / n
    e, b = E.copy(), B.copy()
    acc = np.zeros_like(E)
    for _ in range(n):
        k1 = _stag_rhs(e, b, J, c, L)
        k2 = _stag_rhs(e + 0.5 * dt * k1[0], b + 0.5 * dt * k1[1], J, c, L)
        k3 = _stag_rhs(e + 0.5 * dt * k2[0], b + 0.5 * dt * k2[1], J, c, L)
        k4 = _stag_rhs(e + dt * k3[0], b + dt * k3[1], J, c, L)
        e1 = e + dt / 6 * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0])
        acc += 0.5 * dt * (e + e1)          # trapezoid rule for the time average
        b = b + dt / 6 * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1])
        e = e1
    assert np.abs(Eo - e).max() < 1e-9 * np.abs(e).max()
    assert np.abs(Bo - b).max() < 1e-9 * np.abs(b).max()
    assert np.abs(Ea - acc / tau).max() < 1e-6 * np.abs(Ea).max()


def test_energy_is_conserved_with_particles():
    wl = workloads.weibel(n_particles=20_000, n_cells=32, dt=0.1, steps=60)
    wl.B0 *= 50.0
    st = oracle.State(wl, "emec_psatd")
    rec = st.run(60)
    assert rec["fallbacks"].sum() == 0
    assert np.abs(rec["total"] / rec["total"][0] - 1).max() < 1e-13
    assert rec["field_b"].max() > 1e-6 * rec["total"][0]


def test_boris_limit():
    n, steps, dt = 64, 25, 0.3
    wl = _landau_3v(n=n, b_ext=(0.4, -1.3, 2.0))
    wl.w = np.zeros(n)
    wl.dt = dt
    wl.init_gauss = False
    wl.E0 = np.zeros((3, wl.n_cells))
    wl.B0 = np.zeros((2, wl.n_cells))
    st = oracle.State(wl, "emec_psatd")
    x0, v0 = np.mod(st.x, wl.length), st.v.copy()
    rec = st.run(steps)
    xr, vr = _boris_reference(x0, v0, wl.b_ext, dt, wl.length, steps)
    d = np.abs(st.x - xr)
    assert np.max(np.minimum(d, wl.length - d)) < 1e-12
    assert np.abs(st.v - vr).max() < 1e-12
    assert rec["fallbacks"].sum() == 0


@pytest.mark.slow
def test_weibel_growth_rate():
    """Section 5.3 with the PSATD field solve: the seeded mode grows at the kinetic rate
    within 5 %, energy to 1e-12 (the set-up of the EMEC(LI) pin: 2e5 particles, 64 cells)."""
    wl = workloads.weibel(n_particles=200_000, n_cells=64, dt=0.1, steps=450)
    st = oracle.State(wl, "emec_psatd")
    amp = []
    for _ in range(wl.steps):
        st.run(1)
        amp.append(theory.mode_amplitude(st.B[1], 1))
    t = (np.arange(wl.steps) + 1) * wl.dt
    sel = (t > 15) & (t < 40)
    gamma = np.polyfit(t[sel], np.log(np.array(amp)[sel]), 1)[0]
    ref = theory.weibel_growth(0.5, 0.15, 0.3)
    assert abs(gamma - ref) < 0.05 * ref, (gamma, ref)
    tot = np.array(st.records)["total"]
    assert np.abs(tot / tot[0] - 1).max() < 1e-12
