"""Pins of the oracle's exact charge conservation (section 3.5, eq. (discCont) and eq.
(detbal)): the tent current on the half nodes, deposited and gathered through the pieces of
each particle's path between the tent's kinks, with the charge density on the nodes from
the quadratic B-spline.  Checked against what the mathematics fixes, with the density
computed here by brute force in numpy (every node, every periodic image):

* one particle: rho(x^{n+1}) - rho(x^n) = -(dt/h) D-(j) node by node, for paths that cross
  no half node, one, and many (in both directions and across the periodic boundary);
* a whole run: Gauss' law D- E = rho - mean(rho) holds at every step to rounding, while the
  same run without charge conservation breaks it; energy stays exact;
* the piecewise deposit is the time integral of the tent along the path (fine quadrature);
* physics: Landau damping at the kinetic rate.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from tests import theory


def _b2(t):
    t = np.abs(t)
    return np.where(t < 0.5, 0.75 - t * t, np.where(t < 1.5, 0.5 * (1.5 - t) ** 2, 0.0))


def _rho(x, w, ng, L):
    """rho_i = (1/h) sum_p w_p B2((x_i - x_p)/h) over all periodic images (brute force)."""
    h = L / ng
    xi = np.arange(ng)[:, None] * h
    acc = np.zeros(ng)
    for shift in (-L, 0.0, L):
        acc += (_b2((xi - (np.asarray(x)[None, :] + shift)) / h) * np.asarray(w)[None, :]).sum(1)
    return acc / h


def _dminus(f, h):
    return (f - np.roll(f, 1)) / h


@pytest.mark.parametrize("x0,x1", [(1.23, 1.31), (1.23, 1.61), (1.61, 1.23), (0.4, 3.77),
                                   (3.9, 0.1 + 4.0), (0.05, -0.61), (2.0, 2.0)])
def test_single_particle_continuity(x0, x1):
    ng, L, dt, w = 20, 4.0, 0.3, 0.7
    h = L / ng
    u = (x1 - x0) / dt
    j = oracle.deposit_cc([x0], [x1], [w], [u], ng, h)
    drho = _rho([x1 % L], [w], ng, L) - _rho([x0 % L], [w], ng, L)
    assert np.abs(drho + dt * _dminus(j, h)).max() < 1e-13 * max(1.0, np.abs(drho).max())


def test_piecewise_deposit_is_the_time_average_of_the_tent():
    ng, L, w = 16, 3.2, 1.3
    h = L / ng
    x0, x1 = 0.37, 1.91                       # crosses several half nodes
    j = oracle.deposit_cc([x0], [x1], [w], [1.0], ng, h)
    # time average over the path of the tent at each half node, midpoint rule on 2e5 steps
    s = x0 + (np.arange(200_000) + 0.5) / 200_000 * (x1 - x0)
    xh = (np.arange(ng) + 0.5) * h
    ref = np.zeros(ng)
    for shift in (-L, 0.0, L):
        t = np.abs(xh[:, None] - (s[None, :] + shift)) / h
        ref += np.clip(1.0 - t, 0.0, None).mean(1)
    assert np.abs(j - w * ref / h).max() < 1e-8


def _two_stream(n=4000, ng=32, dt=0.4, steps=60):
    wl = workloads.two_stream(n_particles=n, n_cells=ng, dt=dt, steps=steps, order=1,
                              alpha=0.05, v_beam=3.0, v_spread=0.5)
    return wl


@pytest.mark.parametrize("scheme", ["esec2", "esec1"])
def test_gauss_law_holds_at_every_step(scheme):
    """Fast beams (|v dt| up to ~4 cells per step): the half-node E of the charge-conserving
    run satisfies D- E = rho - mean(rho) after every step to rounding."""
    wl = _two_stream()
    st = oracle.State(wl, scheme, charge_conserving=True)
    h = wl.length / wl.n_cells
    w = np.full(wl.n_particles, wl.length / wl.n_particles)
    worst = 0.0
    st.run(0)
    for _ in range(wl.steps):
        st.run(1)
        rho = _rho(st.x, w, wl.n_cells, wl.length)
        res = _dminus(st.E[0], h) - (rho - rho.mean())
        worst = max(worst, np.abs(res).max() / np.abs(rho - rho.mean()).max())
    assert worst < 1e-12, worst
    # energy is exact up to the first fallback (ESEC1 takes many at this step size)
    rec = np.array(st.records)
    clean = np.cumsum(rec["fallbacks"]) == 0
    assert clean.sum() > 1
    assert np.abs(rec["total"][clean] / rec["total"][0] - 1).max() < 1e-13


def test_without_charge_conservation_gauss_law_drifts():
    """Control: the same run with the node-centred scheme keeps energy but not Gauss' law
    (its spectral divergence of E drifts away from rho - mean(rho))."""
    wl = _two_stream()
    st = oracle.State(wl)
    h = wl.length / wl.n_cells
    w = np.full(wl.n_particles, wl.length / wl.n_particles)
    st.run(wl.steps)
    k = 2 * np.pi * np.fft.fftfreq(wl.n_cells, h)
    dE = np.real(np.fft.ifft(1j * k * np.fft.fft(st.E[0])))
    from_particles = oracle.deposit(1, np.mod(st.x, wl.length), w, np.ones_like(w), wl.n_cells, h)
    res = dE - (from_particles - from_particles.mean())
    assert np.abs(res).max() > 1e-6 * np.abs(from_particles - from_particles.mean()).max()


def test_weighted_3v_run_with_imposed_field():
    wl = workloads.landau_2v(n_particles=3000, n_cells=24, dt=0.3, steps=30)
    wl.w = wl.length / wl.n_particles * (1.0 + 0.5 * workloads.uniforms(4, 9, wl.n_particles))
    wl.b_ext = (0.2, 0.0, 0.7)
    st = oracle.State(wl, charge_conserving=True)
    h = wl.length / wl.n_cells
    rec = st.run(30)
    rho = _rho(st.x, wl.w, wl.n_cells, wl.length)
    assert np.abs(_dminus(st.E[0], h) - (rho - rho.mean())).max() < 1e-12 * np.abs(rho).max()
    assert np.abs(rec["total"] / rec["total"][0] - 1).max() < 1e-13


def test_rejected_outside_its_scope():
    wl = _two_stream(n=100, steps=1)
    wl.order = 2
    with pytest.raises(ValueError):
        oracle.State(wl, charge_conserving=True).run(1)


@pytest.mark.slow
def test_landau_damping_rate():
    k = 0.5
    wl = workloads.landau(quiet=True, steps=130)
    st = oracle.State(wl, charge_conserving=True)
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
    assert abs(math.pi / np.mean(np.diff(t[pk])) - w.real) < 0.03 * w.real
