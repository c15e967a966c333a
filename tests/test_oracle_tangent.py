"""Pins of the oracle's derivative (the reference gradient for the adjoint form).

The tangent-linear run of the oracle is checked against things other than itself:
central finite differences of the oracle's own forward run (FP64), finite differences of
the independent 50-digit reference with a step far below FP64 resolution, and the
derivative of the inverse-CDF sampling against finite differences of the sampler.
"""
import numpy as np
import pytest

import oracle
import workloads
from oracle import mp_reference as mpr


def _small_two_stream(n=240, ng=16, steps=30, order=2, alphas=(0.02, 0.01, 0.005), seed=11):
    return workloads.adjoint_two_stream(n_particles=n, n_cells=ng, alphas=alphas,
                                        v_beam=1.2, v_spread=0.3, dt=0.1, steps=steps,
                                        order=order, seed=seed)


def test_sampling_tangent_matches_finite_differences():
    """dx/dalpha_m of the inverse-CDF positions (implicit differentiation) against
    central differences of the Newton sampler at fixed uniforms."""
    wl = _small_two_stream(n=500)
    u = wl.meta["u"]
    modes = wl.meta["modes"]
    T = oracle.density_mode_tangents(wl.x, modes)
    for m in range(len(modes)):
        eps = 1e-6
        up = [(k, a + (eps if j == m else 0.0)) for j, (k, a) in enumerate(modes)]
        dn = [(k, a - (eps if j == m else 0.0)) for j, (k, a) in enumerate(modes)]
        fd = (workloads.sample_density(u, wl.length, up)
              - workloads.sample_density(u, wl.length, dn)) / (2 * eps)
        assert np.abs(fd - T[m]).max() < 1e-6 * np.abs(T[m]).max() + 1e-9


def test_tlm_forward_part_is_the_oracle_run():
    """The state the tangent-linear run carries is the oracle's ordinary run, bit for bit."""
    wl = _small_two_stream()
    out = oracle.tlm_run(wl, 25, np.zeros((0, wl.n_particles)), np.zeros((0, wl.n_particles)), 1.0)
    st = oracle.State(wl)
    rec = st.run(25)
    assert np.array_equal(out["x"], st.x) and np.array_equal(out["v"], st.v[0])
    assert np.array_equal(out["E"], st.E[0])
    assert np.array_equal(out["records"]["total"], rec["total"])
    assert abs(out["J"] - 1.0 * rec["field_e"][1:].sum()) < 1e-14 * out["J"]


@pytest.mark.parametrize("order", [1, 2])
def test_tlm_matches_fp64_central_differences(order):
    """dJ and the final tangents along random directions against central differences
    of the oracle's FP64 forward run (Gauss start included).  Step 1e-5: the difference
    quotient's rounding error (~1e-16 |J| / step) then sits well below the tolerance,
    and its truncation error (~step^2) too."""
    wl = _small_two_stream(order=order)
    n, steps = wl.n_particles, 30
    rng = np.random.default_rng(5)
    K = 3
    dx = rng.normal(size=(K, n)) * 0.05
    dv = rng.normal(size=(K, n)) * 0.05
    out = oracle.tlm_run(wl, steps, dx, dv, wl.dt)
    assert out["records"]["fallbacks"].sum() == 0
    eps = 1e-5
    for k in range(K):
        res = []
        for sgn in (1, -1):
            w2 = _small_two_stream(order=order)
            w2.x = wl.x + sgn * eps * dx[k]
            w2.v = wl.v + sgn * eps * dv[k][None, :]
            res.append(oracle.tlm_run(w2, steps, np.zeros((0, n)), np.zeros((0, n)), wl.dt))
        fdJ = (res[0]["J"] - res[1]["J"]) / (2 * eps)
        assert abs(fdJ - out["dJ"][k]) < 1e-7 * np.abs(out["dJ"]).max(), (k, fdJ, out["dJ"][k])
        fdv = (res[0]["v"] - res[1]["v"]) / (2 * eps)
        assert np.abs(fdv - out["dv"][k]).max() < 1e-6 * np.abs(out["dv"][k]).max()
        fdx = (res[0]["x"] - res[1]["x"]) / (2 * eps)
        fdx = fdx - wl.length * np.round(fdx * 2 * eps / wl.length) / (2 * eps)
        assert np.abs(fdx - out["dx"][k]).max() < 1e-6 * np.abs(out["dx"][k]).max()
        fdE = (res[0]["E"] - res[1]["E"]) / (2 * eps)
        assert np.abs(fdE - out["dE"][k]).max() < 1e-6 * np.abs(out["dE"][k]).max()


@pytest.mark.parametrize("order", [1, 2])
def test_tlm_matches_50_digit_differences(order):
    """A few particles, given E^0 and a tangent of E^0: the FP64 tangent-linear state
    after 4 steps against central differences of the independent 50-digit reference
    with step 1e-20 (truncation ~1e-40), to 1e-11."""
    import mpmath as mp
    ng, L, dt, steps = 8, 2.0, 0.35, 4
    x = np.array([0.13, 0.61, 1.07, 1.72])
    v = np.array([0.9, -0.4, 0.25, -1.1])
    w = np.full(4, L / 4)
    E0 = np.array([0.1, -0.05, 0.2, 0.0, -0.15, 0.05, -0.1, -0.05])
    tx = np.array([0.3, -0.2, 0.5, 0.1])
    tv = np.array([-0.4, 0.7, 0.2, -0.3])
    tE = np.array([0.05, 0.1, -0.2, 0.15, -0.05, 0.0, 0.1, -0.15])
    wl = workloads.Workload(name="tiny", nv=1, scheme="esec2", order=order, n_cells=ng,
                            length=L, dt=dt, steps=steps, x=x.copy(), v=v[None, :].copy(),
                            E0=np.stack([E0, np.zeros(ng), np.zeros(ng)]), init_gauss=False)
    out = oracle.tlm_run(wl, steps, tx[None, :], tv[None, :], 1.0, dE=tE[None, :])
    eps = mp.mpf("1e-20")

    def run(sgn):
        xs = [mp.mpf(a) + sgn * eps * mp.mpf(b) for a, b in zip(x, tx)]
        vs = [mp.mpf(a) + sgn * eps * mp.mpf(b) for a, b in zip(v, tv)]
        Es = [mp.mpf(a) + sgn * eps * mp.mpf(b) for a, b in zip(E0, tE)]
        st = mpr.MPState(1, "esec2", order, ng, L, dt, xs, [vs], list(w), [Es, [0] * ng, [0] * ng])
        J = mp.mpf(0)
        for _ in range(steps):
            st.step()
            J += st.energy()[1]
        assert st.fallbacks == 0
        return st, J
    a, Ja = run(1)
    b, Jb = run(-1)
    fdv = np.array([float((p - q) / (2 * eps)) for p, q in zip(a.v[0], b.v[0])])
    fdE = np.array([float((p - q) / (2 * eps)) for p, q in zip(a.E[0], b.E[0])])
    fdx = []
    for p, q in zip(a.x, b.x):
        d = p - q
        d -= L * mp.nint(d / L)
        fdx.append(float(d / (2 * eps)))
    fdx = np.array(fdx)
    fdJ = float((Ja - Jb) / (2 * eps))
    sc = max(np.abs(fdv).max(), np.abs(fdx).max())
    assert np.abs(out["dv"][0] - fdv).max() < 1e-11 * sc
    assert np.abs(out["dx"][0] - fdx).max() < 1e-11 * sc
    assert np.abs(out["dE"][0] - fdE).max() < 1e-11 * np.abs(fdE).max()
    assert abs(out["dJ"][0] - fdJ) < 1e-11 * abs(fdJ)


def test_two_stream_gradient_matches_parameter_differences():
    """The parameter gradient (mode amplitudes, beam speed, beam spread) of a small
    two-stream run against central differences of regenerated workloads: the sampling
    derivative, the Gauss start and the steps together."""
    alphas = (0.02, 0.01, 0.005)
    kw = dict(n_particles=300, n_cells=16, v_spread=0.3, dt=0.1, steps=40, order=2, seed=13)
    wl = workloads.adjoint_two_stream(alphas=alphas, v_beam=1.2, **kw)
    J, dJ, out = oracle.two_stream_gradient(wl, 40)
    assert out["records"]["fallbacks"].sum() == 0
    eps = 1e-7

    def loss(al, vb, vs):
        w2 = workloads.adjoint_two_stream(alphas=al, v_beam=vb, **dict(kw, v_spread=vs))
        n = w2.n_particles
        return oracle.tlm_run(w2, 40, np.zeros((0, n)), np.zeros((0, n)), w2.dt)["J"]
    fd = []
    for m in range(len(alphas)):
        up = list(alphas); up[m] += eps
        dn = list(alphas); dn[m] -= eps
        fd.append((loss(up, 1.2, 0.3) - loss(dn, 1.2, 0.3)) / (2 * eps))
    fd.append((loss(alphas, 1.2 + eps, 0.3) - loss(alphas, 1.2 - eps, 0.3)) / (2 * eps))
    fd.append((loss(alphas, 1.2, 0.3 + eps) - loss(alphas, 1.2, 0.3 - eps)) / (2 * eps))
    fd = np.array(fd)
    assert np.abs(fd - dJ).max() < 1e-5 * np.abs(dJ).max(), (fd, dJ)
