"""Pins of the oracle's EMEC(LF) (section 4.1, eq. (EMleapfrog)): the Yee leapfrog with B at
half steps and the non-standard magnetic energy W_B^n = c^2/2 h sum B^{n+1/2} . B^{n-1/2},
against what the mathematics fixes independently of the oracle's code:

* vacuum: a travelling wave of either polarisation follows the leapfrog's own dispersion
  relation sin(w dt/2) = (c dt/h) sin(k h/2), with B = E / c, for many steps, and the
  energy W_E + W_B is then exactly constant;
* at the magic step c dt = h the relation is the exact light-wave relation w = c k;
* energy with particles to 1e-13 (the energy identity of section 4.1);
* the Boris limit and the Weibel growth rate.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from tests import theory
from tests.test_oracle_pins import _boris_reference, _landau_3v

S = "emec_lf"


def _vacuum(ng, L, c, dt, m, pol):
    """Workload with zero-weight particles and the leapfrog's travelling wave of mode m at
    t = 0 (E on the nodes at t = 0, B on the half nodes at t = -dt/2)."""
    h = L / ng
    xn, xh = np.arange(ng) * h, (np.arange(ng) + 0.5) * h
    k = 2 * math.pi * m / L
    w = 2.0 / dt * math.asin(c * dt / h * math.sin(0.5 * k * h))
    wl = _landau_3v(n=4, b_ext=(0.0, 0.0, 0.0))
    wl.n_cells, wl.length, wl.dt, wl.c = ng, L, dt, c
    wl.x = np.linspace(0.1, L - 0.1, 4)
    wl.w = np.zeros(4)
    wl.init_gauss = False
    wl.E0 = np.zeros((3, ng))
    wl.B0 = np.zeros((2, ng))
    if pol == 0:     # E_y = c B_z
        wl.E0[1], wl.B0[1] = np.cos(k * xn), np.cos(k * xh + 0.5 * w * dt) / c
    else:            # E_z = -c B_y
        wl.E0[2], wl.B0[0] = np.cos(k * xn), -np.cos(k * xh + 0.5 * w * dt) / c
    return wl, k, w, xn, xh


@pytest.mark.parametrize("m,pol", [(1, 0), (7, 1), (20, 0)])
def test_vacuum_wave_follows_the_leapfrog_dispersion(m, pol):
    ng, L, c, dt, steps = 64, 4 * math.pi, 1.0, 0.15, 150
    wl, k, w, xn, xh = _vacuum(ng, L, c, dt, m, pol)
    st = oracle.State(wl, S)
    rec = st.run(steps)
    t = steps * dt
    ec, bc, sg = (1, 1, 1.0) if pol == 0 else (2, 0, -1.0)
    assert np.abs(st.E[ec] - np.cos(k * xn - w * t)).max() < 1e-11
    assert np.abs(st.B[bc] - sg * np.cos(k * xh - w * (t - 0.5 * dt)) / c).max() < 1e-11
    assert np.abs(rec["total"] / rec["total"][0] - 1).max() < 1e-13


def test_magic_time_step_gives_exact_light_waves():
    """c dt = h: sin(w dt/2) = sin(k h/2), so w = c k for every mode."""
    ng, L, c = 32, 2 * math.pi, 1.0
    dt = L / ng / c
    wl, k, w, xn, xh = _vacuum(ng, L, c, dt, 5, 0)
    assert abs(w - c * k) < 1e-12
    st = oracle.State(wl, S)
    st.run(64)
    assert np.abs(st.E[1] - np.cos(k * xn - c * k * 64 * dt)).max() < 1e-11


def test_energy_is_conserved_with_particles():
    wl = workloads.weibel(n_particles=20_000, n_cells=32, dt=0.1, steps=60)
    wl.B0 *= 50.0
    st = oracle.State(wl, S)
    rec = st.run(60)
    assert rec["fallbacks"].sum() == 0
    assert np.abs(rec["total"] / rec["total"][0] - 1).max() < 1e-13
    assert rec["field_b"].max() > 1e-6 * rec["total"][0]


def test_magnetic_energy_is_the_leapfrog_product():
    """Record 0 of a run from B^{-1/2} = B holds c^2/2 h sum B^{1/2} . B^{-1/2}, with
    B^{1/2} = B^{-1/2} - dt curl E^0 written out here with numpy differences."""
    ng, L, c, dt = 16, 3.0, 0.7, 0.05
    h = L / ng
    rng = np.random.default_rng(2)
    wl = _landau_3v(n=4, b_ext=(0.0, 0.0, 0.0))
    wl.n_cells, wl.length, wl.dt, wl.c = ng, L, dt, c
    wl.x = np.linspace(0.1, L - 0.1, 4)
    wl.w = np.zeros(4)
    wl.init_gauss = False
    wl.E0 = rng.normal(size=(3, ng))
    wl.B0 = rng.normal(size=(2, ng))
    st = oracle.State(wl, S)
    rec = st.run(0)
    dp = lambda f: (np.roll(f, -1) - f) / h     # noqa: E731  nodes -> half nodes
    b_half = np.stack([wl.B0[0] + dt * dp(wl.E0[2]), wl.B0[1] - dt * dp(wl.E0[1])])
    wb = 0.5 * c * c * h * np.sum(b_half * wl.B0)
    assert abs(rec["field_b"][0] - wb) < 1e-13 * abs(wb)
    assert abs(rec["field_e"][0] - 0.5 * h * np.sum(wl.E0 ** 2)) < 1e-13 * rec["field_e"][0]


def test_boris_limit():
    n, steps, dt = 64, 25, 0.3
    wl = _landau_3v(n=n, b_ext=(0.4, -1.3, 2.0))
    wl.w = np.zeros(n)
    wl.dt = dt
    wl.init_gauss = False
    wl.E0 = np.zeros((3, wl.n_cells))
    wl.B0 = np.zeros((2, wl.n_cells))
    st = oracle.State(wl, S)
    x0, v0 = np.mod(st.x, wl.length), st.v.copy()
    rec = st.run(steps)
    xr, vr = _boris_reference(x0, v0, wl.b_ext, dt, wl.length, steps)
    d = np.abs(st.x - xr)
    assert np.max(np.minimum(d, wl.length - d)) < 1e-12
    assert np.abs(st.v - vr).max() < 1e-12
    assert rec["fallbacks"].sum() == 0


@pytest.mark.slow
def test_weibel_growth_rate():
    """Section 5.3 with the leapfrog field update (2e5 particles, 64 cells, dt 0.1: c dt/h =
    0.51): the seeded mode grows at the kinetic rate within 5 %, energy to 1e-12."""
    wl = workloads.weibel(n_particles=200_000, n_cells=64, dt=0.1, steps=450)
    st = oracle.State(wl, S)
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
