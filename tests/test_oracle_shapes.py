"""Pins of the oracle's building blocks against textbook properties (no GPU).

Shape functions (section 2.2): B-splines are a partition of unity with zero first moment;
the degree-2 spline has constant second moment 1/4 (variance of three convolved unit
boxes), the tent has d(1-d).  Deposit and gather with one shape are adjoint (the
identity used in eq. (brokenEcons)).  The spectral Gauss solve reproduces the closed-form
field of a single Fourier mode.  The Crank-Nicolson solve satisfies its own system and,
in vacuum, rotates each Fourier mode by the Cayley angle 2 atan(c k' dt / 2).
"""
import math

import numpy as np
import pytest

import oracle

rng = np.random.default_rng(12345)


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("shift", [0.0, 0.5])
def test_partition_of_unity_and_moments(order, shift):
    ng, L = 16, 7.3
    h = L / ng
    for pos in np.concatenate([rng.uniform(-0.3 * L, 1.3 * L, 400),
                               np.arange(-2, 2 * ng + 2) * 0.5 * h]):
        idx, wt = oracle.stencil(order, pos, h, ng, shift)
        assert abs(wt.sum() - 1.0) < 1e-14
        assert np.all(wt > 0) and np.all((idx >= 0) & (idx < ng))
        # moments about the particle, using the unwrapped node nearest in image
        xi = pos / h - shift
        nodes = np.array([j for j in range(int(math.floor(xi)) - 1, int(math.floor(xi)) + 3)
                          if (j % ng) in idx and abs(j - xi) < (order + 1) / 2])
        d = nodes - xi
        w = np.array([wt[list(idx).index(j % ng)] for j in nodes])
        assert abs(np.sum(w * d)) < 1e-13
        if order == 2:
            assert abs(np.sum(w * d * d) - 0.25) < 1e-13
        else:
            f = xi - math.floor(xi)
            assert abs(np.sum(w * d * d) - f * (1 - f)) < 1e-13


def test_shape_values():
    h, ng = 1.0, 10
    idx, wt = oracle.stencil(1, 3.3, h, ng)
    assert dict(zip(idx, wt)) == pytest.approx({3: 0.7, 4: 0.3}, abs=1e-15)
    idx, wt = oracle.stencil(2, 5.0, h, ng)
    assert dict(zip(idx, wt)) == pytest.approx({4: 0.125, 5: 0.75, 6: 0.125}, abs=1e-15)
    idx, wt = oracle.stencil(2, 5.5, h, ng)           # half-integer tie: two nodes
    assert dict(zip(idx, wt)) == pytest.approx({5: 0.5, 6: 0.5}, abs=1e-15)
    idx, wt = oracle.stencil(1, 9.75, h, ng)          # periodic wrap to node 0
    assert dict(zip(idx, wt)) == pytest.approx({9: 0.25, 0: 0.75}, abs=1e-15)


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("shift", [0.0, 0.5])
def test_deposit_gather_adjoint(order, shift):
    ng, L, n = 24, 5.0, 3000
    h = L / ng
    x = rng.uniform(-0.1 * L, 1.1 * L, n)
    w = rng.uniform(0.5, 1.5, n)
    u = rng.normal(size=n)
    F = rng.normal(size=ng)
    j = oracle.deposit(order, x, w, u, ng, h, shift)
    Fp = oracle.gather(order, x, F, h, shift)
    lhs = np.sum(w * u * Fp)
    rhs = h * np.sum(F * j)
    assert abs(lhs - rhs) <= 1e-13 * np.sum(np.abs(w * u * Fp))
    # charge: sum_i h rho_i = sum_p w_p
    rho = oracle.deposit(order, x, w, np.ones(n), ng, h, shift)
    assert abs(h * rho.sum() - w.sum()) < 1e-12 * w.sum()


@pytest.mark.parametrize("ng,m,alpha", [(32, 1, 0.05), (64, 3, 0.2), (33, 5, 0.1)])
def test_gauss_single_mode(ng, m, alpha):
    # one particle on each node with CIC gives rho_i = w_i / h exactly
    L = 2 * math.pi / 0.5
    h = L / ng
    k = 2 * math.pi * m / L
    xi = np.arange(ng) * h
    w = h * (1 + alpha * np.cos(k * xi))
    E = oracle.gauss(1, xi, w, ng, L)
    # dE/dx = rho - 1 = alpha cos(k x)  ->  E = (alpha / k) sin(k x), zero mean
    assert np.max(np.abs(E - alpha / k * np.sin(k * xi))) < 1e-13
    assert abs(E.sum()) < 1e-12


def _apply_cn(y, h, s):
    lap = (np.roll(y, -1) - 2 * y + np.roll(y, 1)) / h ** 2
    return y - s * lap


@pytest.mark.parametrize("ng", [16, 37, 256])
def test_cn_solve_residual(ng):
    h, s = 0.07, 0.3 ** 2
    r = rng.normal(size=ng)
    y = oracle.cn_solve(ng, h, s, r)
    assert np.max(np.abs(_apply_cn(y, h, s) - r)) < 1e-12 * np.max(np.abs(r))


def test_cn_vacuum_light_wave():
    """Vacuum (zero-weight particles): E_y = cos(k x), B_z = 0 rotates by the CN angle."""
    from workloads import Workload
    ng, L, dt, c, m = 64, 4 * math.pi, 0.2, 1.0, 3
    h = L / ng
    k = 2 * math.pi * m / L
    kd = 2 / h * math.sin(k * h / 2)          # symbol of the staggered differences
    theta = 2 * math.atan(0.5 * dt * c * kd)
    xi = np.arange(ng) * h
    E0 = np.zeros((3, ng))
    E0[1] = np.cos(k * xi)
    wl = Workload(name="vacuum", nv=3, scheme="emec_li", order=2, n_cells=ng, length=L,
                  dt=dt, steps=10, x=np.array([0.3, 1.7]), v=np.zeros((3, 2)), c=c,
                  w=np.zeros(2), E0=E0, B0=np.zeros((2, ng)), init_gauss=False)
    st = oracle.State(wl)
    rec = st.run(10)
    assert np.max(np.abs(st.E[1] - math.cos(10 * theta) * np.cos(k * xi))) < 1e-12
    te = rec["total"]
    assert np.max(np.abs(te - te[0])) < 1e-13 * te[0]
