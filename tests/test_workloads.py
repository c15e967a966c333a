"""The seeded input generators: determinism, ranges and the sampled distributions."""
import math

import numpy as np

import workloads
from workloads import generators as g


def test_counter_based_and_deterministic():
    a = workloads.uniforms(11, 1, 1000)
    b = workloads.uniforms(11, 1, 1000)
    assert np.array_equal(a, b)
    assert np.array_equal(workloads.uniforms(11, 1, 100, offset=900), a[900:])
    assert not np.array_equal(workloads.uniforms(12, 1, 1000), a)
    assert not np.array_equal(workloads.uniforms(11, 2, 1000), a)
    assert a.min() > 0.0 and a.max() < 1.0
    # first value of the SplitMix64 finaliser at a fixed input (pins the constants)
    z = g._mix64(np.array([1], dtype=np.uint64))[0]
    assert int(z) == 0x5692161D100B05E5


def test_normal_moments():
    x = workloads.normals(3, 2, 400_000)
    assert abs(x.mean()) < 0.01 and abs(x.std() - 1) < 0.01
    q = g.quiet_normals(1 << 16)
    assert abs(q.mean()) < 1e-3 and abs(q.std() - 1) < 1e-3


def test_inverse_cdf_density():
    L, k, a = 4 * math.pi, 0.5, 0.3
    u = (np.arange(200_000) + 0.5) / 200_000
    x = workloads.sample_density(u, L, [(k, a)])
    assert x.min() >= 0 and x.max() < L
    # exact CDF at the samples equals u
    F = (x + a / k * np.sin(k * x)) / L
    assert np.max(np.abs(F - u)) < 1e-14
    hist, edges = np.histogram(x, bins=40, range=(0, L))
    c = 0.5 * (edges[1:] + edges[:-1])
    dens = hist / (len(x) * (L / 40)) * L
    assert np.max(np.abs(dens - (1 + a * np.cos(k * c)))) < 0.02


def test_workload_shapes():
    wl = workloads.two_stream(n_particles=1000, n_cells=64)
    assert wl.v.shape == (1, 1000) and wl.order == 2 and wl.scheme == "esec2"
    assert np.all(np.sign(wl.v[0][::2]) > 0) and np.all(np.sign(wl.v[0][1::2]) < 0)
    wb = workloads.weibel(n_particles=1000, n_cells=16)
    assert wb.v.shape == (3, 1000) and wb.B0.shape == (2, 16) and not wb.init_gauss
    assert abs(wb.B0[1].max() - 1e-3) < 1e-4
    runs = workloads.batched_landau(n_runs=16, np_scale=1e-2, steps=5)
    assert len(runs) == 16
    assert all(r.n_cells in (32, 64, 128, 256, 512) for r in runs)
    assert all(100 <= r.n_particles <= 10_000 for r in runs)
    assert all(0.3 <= r.meta["k"] <= 0.6 for r in runs)
