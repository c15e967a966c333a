"""Seeded, synthetic particle-in-cell inputs.

Random numbers come from a counter-based SplitMix64: the i-th draw of stream ``s`` under
seed ``q`` is ``mix64(key(q, s) + (i + 1) * GAMMA)``, where ``mix64`` is Steele, Lea and
Flood's SplitMix64 finaliser.  Draws therefore do not depend on the numpy version, and any
sub-range can be regenerated on its own.  Positions are drawn by inverting the cumulative
distribution of a periodic density ``1 + sum_m alpha_m cos(k_m x)`` with Newton's method;
velocities are Gaussian (Box-Muller on two independent uniform streams).

The workloads follow the paper's test problems recast to one spatial dimension: linear
Landau damping (section 5.1), the two-stream instability (section 5.2) and the Weibel
instability (section 5.3), plus a batch of independent Landau runs and the two-stream
set-up used for gradients.  Sizes are parameters so tests can run small variants.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_STREAM = np.uint64(0xD1B54A32D192ED03)
_CHUNK = 1 << 22

# Stream identifiers, one per independent quantity.
S_POS, S_VX, S_VY, S_VZ, S_AUX = 1, 2, 4, 6, 8


def _mix64(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _key(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        base = np.array([np.uint64(seed & 0xFFFFFFFFFFFFFFFF) * GAMMA
                         + np.uint64(stream) * _STREAM + np.uint64(1)], dtype=np.uint64)
        return _mix64(base)[0]


def uniforms(seed: int, stream: int, n: int, offset: int = 0) -> np.ndarray:
    """``n`` doubles in the open interval (0, 1), draws ``offset .. offset+n-1``."""
    out = np.empty(n, dtype=np.float64)
    k = _key(seed, stream)
    with np.errstate(over="ignore"):
        for a in range(0, n, _CHUNK):
            b = min(n, a + _CHUNK)
            i = np.arange(offset + a + 1, offset + b + 1, dtype=np.uint64)
            z = _mix64(k + i * GAMMA)
            out[a:b] = ((z >> np.uint64(11)).astype(np.float64) + 0.5) * (2.0 ** -53)
    return out


def normals(seed: int, stream: int, n: int, offset: int = 0) -> np.ndarray:
    """Standard normal draws by Box-Muller from streams ``stream`` and ``stream + 1``."""
    u1 = uniforms(seed, stream, n, offset)
    u2 = uniforms(seed, stream + 1, n, offset)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


def radical_inverse2(n: int) -> np.ndarray:
    """Base-2 radical inverse (van der Corput) of ``0 .. n-1``, shifted to cell centres."""
    i = np.arange(n, dtype=np.uint64)
    r = np.zeros(n, dtype=np.float64)
    f = 0.5
    while np.any(i):
        r += f * (i & np.uint64(1)).astype(np.float64)
        i >>= np.uint64(1)
        f *= 0.5
    return r + 0.5 / (1 << max(1, int(math.ceil(math.log2(max(n, 2))))))


def quiet_normals(n: int) -> np.ndarray:
    """Deterministic standard-normal values: the inverse normal CDF of the bit-reversed
    stratified sequence, so that consecutive particles sample the whole distribution."""
    from scipy.special import ndtri
    return ndtri(radical_inverse2(n))


def sample_density(u: np.ndarray, length: float,
                   modes: Sequence[Tuple[float, float]]) -> np.ndarray:
    """Inverse-CDF positions for the density ``1 + sum alpha cos(k x)`` on ``[0, L)``.

    ``modes`` is a list of ``(k, alpha)`` with every ``k L`` a multiple of ``2 pi`` and
    ``sum |alpha| < 1``.  Solves ``x + sum (alpha/k) sin(k x) = u L`` to ``1e-15 L``.
    """
    x = u * length
    target = u * length
    if not modes:
        return x
    assert sum(abs(a) for _, a in modes) < 1.0
    for _ in range(60):
        f = x - target
        d = np.ones_like(x)
        for k, a in modes:
            f = f + (a / k) * np.sin(k * x)
            d = d + a * np.cos(k * x)
        step = f / d
        x = x - step
        if np.max(np.abs(step)) < 1e-15 * length:
            break
    x = np.where(x >= length, x - length, x)
    x = np.where(x < 0.0, x + length, x)
    return x


@dataclasses.dataclass
class Workload:
    """One run: discretisation parameters plus the initial particle and field arrays."""

    name: str
    nv: int                 # velocity components per particle: 1 or 3
    scheme: str             # "esec2", "esec1" or "emec_li"
    order: int              # B-spline degree of the shape function: 1 (tent) or 2
    n_cells: int
    length: float
    dt: float
    steps: int
    x: np.ndarray           # [N_p] positions in [0, L)
    v: np.ndarray           # [nv, N_p] velocities
    c: float = 1.0
    b_ext: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    w: Optional[np.ndarray] = None       # None: uniform weights L / N_p
    E0: Optional[np.ndarray] = None      # [3, N_g] node field; None with init_gauss
    B0: Optional[np.ndarray] = None      # [2, N_g] (B_y, B_z) at half nodes (EM)
    init_gauss: bool = True
    meta: Dict = dataclasses.field(default_factory=dict)

    @property
    def n_particles(self) -> int:
        return int(self.x.shape[0])


def landau(n_particles: int = 100_000, n_cells: int = 64, k: float = 0.5,
           alpha: float = 0.01, dt: float = 0.1, steps: int = 200, order: int = 1,
           seed: int = 1, scheme: str = "esec2", quiet: bool = False) -> Workload:
    """1D-1V linear Landau damping: density ``1 + alpha cos(k x)``, ``v ~ N(0, 1)``.

    ``quiet`` is a phase-space quiet start: positions from the stratified points
    ``(p + 1/2) / N_p`` (inverse-CDF mapped) and velocities from ``quiet_normals``.
    """
    length = 2.0 * math.pi / k
    if quiet:
        u = (np.arange(n_particles, dtype=np.float64) + 0.5) / n_particles
        v = quiet_normals(n_particles)[None, :]
    else:
        u = uniforms(seed, S_POS, n_particles)
        v = normals(seed, S_VX, n_particles)[None, :]
    x = sample_density(u, length, [(k, alpha)])
    return Workload(name="landau", nv=1, scheme=scheme, order=order, n_cells=n_cells,
                    length=length, dt=dt, steps=steps, x=x, v=v,
                    meta=dict(k=k, alpha=alpha, seed=seed, quiet=quiet))


def two_stream(n_particles: int = 10_000_000, n_cells: int = 512, k: float = 0.2,
               alpha: float = 1e-3, v_beam: float = 3.0, v_spread: float = 0.1,
               dt: float = 0.05, steps: int = 2000, order: int = 2, seed: int = 2,
               scheme: str = "esec2", modes: Optional[Sequence[Tuple[float, float]]] = None,
               quiet: bool = False) -> Workload:
    """1D-1V two-stream: beams at ``+-v_beam`` (even particles +, odd -), density
    ``1 + alpha cos(k x)`` (or the given ``modes``), thermal spread ``v_spread``.

    ``quiet`` gives each beam stratified positions and ``quiet_normals`` spreads."""
    length = 2.0 * math.pi / k
    sign = np.where(np.arange(n_particles) % 2 == 0, 1.0, -1.0)
    if quiet:
        half = (n_particles + 1) // 2
        q = (np.arange(half, dtype=np.float64) + 0.5) / half
        u = np.repeat(q, 2)[:n_particles]
        g = np.repeat(quiet_normals(half), 2)[:n_particles]
    else:
        u = uniforms(seed, S_POS, n_particles)
        g = normals(seed, S_VX, n_particles)
    x = sample_density(u, length, list(modes) if modes is not None else [(k, alpha)])
    v = (v_beam * sign + v_spread * g)[None, :]
    return Workload(name="two_stream", nv=1, scheme=scheme, order=order,
                    n_cells=n_cells, length=length, dt=dt, steps=steps, x=x, v=v,
                    meta=dict(k=k, alpha=alpha, v_beam=v_beam, v_spread=v_spread,
                              seed=seed, quiet=quiet, u=u, g=g, sign=sign))


def weibel(n_particles: int = 20_000_000, n_cells: int = 256, k0: float = 0.5,
           vth_x: float = 0.15, vth_perp: float = 0.3, b_seed: float = 1e-3,
           c: float = 1.0, dt: float = 0.05, steps: int = 1000, order: int = 2,
           seed: int = 3) -> Workload:
    """1D-3V Weibel: quiet-start positions ``(p + 1/2) L / N_p``, bi-Maxwellian
    velocities, ``E = 0`` and ``B_z = b sin(k0 x)`` sampled at the half nodes."""
    length = 2.0 * math.pi / k0
    x = (np.arange(n_particles, dtype=np.float64) + 0.5) * (length / n_particles)
    v = np.stack([vth_x * normals(seed, S_VX, n_particles),
                  vth_perp * normals(seed, S_VY, n_particles),
                  vth_perp * normals(seed, S_VZ, n_particles)])
    h = length / n_cells
    xh = (np.arange(n_cells, dtype=np.float64) + 0.5) * h
    B0 = np.zeros((2, n_cells))
    B0[1] = b_seed * np.sin(k0 * xh)
    return Workload(name="weibel", nv=3, scheme="emec_li", order=order, n_cells=n_cells,
                    length=length, dt=dt, steps=steps, x=x, v=v, c=c,
                    E0=np.zeros((3, n_cells)), B0=B0, init_gauss=False,
                    meta=dict(k0=k0, vth_x=vth_x, vth_perp=vth_perp, b_seed=b_seed,
                              seed=seed))


def landau_2v(n_particles: int = 100_000, n_cells: int = 64, dt: float = 0.1,
              steps: int = 200, order: int = 1, alpha: float = 0.01, seed: int = 1,
              scheme: str = "esec2") -> Workload:
    """Landau damping with two velocity components (the paper's tests have a 2D velocity
    space, section 5): the 1D-1V Landau workload plus a thermal v_y ~ N(0, 1), v_z = 0, no
    magnetic field, run as 1D-3V."""
    wl = landau(n_particles=n_particles, n_cells=n_cells, dt=dt, steps=steps, order=order,
                alpha=alpha, seed=seed, scheme=scheme)
    wl.v = np.stack([wl.v[0], normals(seed, S_VY, n_particles), np.zeros(n_particles)])
    wl.nv = 3
    wl.name = "landau_2v"
    return wl


def _run_seed(seed: int, r: int) -> int:
    with np.errstate(over="ignore"):
        z = _mix64(np.array([np.uint64(seed) * GAMMA + np.uint64(r + 1) * _STREAM],
                            dtype=np.uint64))[0]
    return int(z & np.uint64(0x7FFFFFFFFFFFFFFF))


def batched_landau(n_runs: int = 512, seed: int = 4, log10_np: Tuple[float, float] = (4.0, 6.0),
                   cells: Sequence[int] = (32, 64, 128, 256, 512),
                   k_range: Tuple[float, float] = (0.3, 0.6),
                   alpha_range: Tuple[float, float] = (1e-3, 5e-2),
                   dt: float = 0.1, steps: int = 500, order: int = 1,
                   np_scale: float = 1.0) -> List[Workload]:
    """An ensemble of independent 1D-1V Landau runs with uneven sizes.

    Run ``r`` draws its cell count, particle count (log-uniform), wavenumber and
    amplitude from the batch seed, then its particles from its own derived seed.
    ``np_scale`` shrinks every particle count (for small test variants).
    """
    uc = uniforms(seed, S_AUX, n_runs)
    un = uniforms(seed, S_AUX + 1, n_runs)
    uk = uniforms(seed, S_AUX + 2, n_runs)
    ua = uniforms(seed, S_AUX + 3, n_runs)
    runs = []
    for r in range(n_runs):
        ng = int(cells[min(len(cells) - 1, int(uc[r] * len(cells)))])
        npart = max(1, int(round(np_scale * 10.0 ** (log10_np[0] + (log10_np[1] - log10_np[0]) * un[r]))))
        k = k_range[0] + (k_range[1] - k_range[0]) * uk[r]
        a = alpha_range[0] + (alpha_range[1] - alpha_range[0]) * ua[r]
        wl = landau(n_particles=npart, n_cells=ng, k=k, alpha=a, dt=dt, steps=steps,
                    order=order, seed=_run_seed(seed, r))
        wl.name = f"landau_run{r}"
        runs.append(wl)
    return runs


def adjoint_two_stream(n_particles: int = 1_000_000, n_cells: int = 256, k: float = 0.2,
                       alphas: Sequence[float] = (1e-3,) * 8, v_beam: float = 3.0,
                       v_spread: float = 0.1, dt: float = 0.05, steps: int = 500,
                       order: int = 2, seed: int = 5) -> Workload:
    """Two-stream with density ``1 + sum_m alpha_m cos(m k x)``, ``m = 1 .. len(alphas)``.

    ``meta`` keeps the beam signs and the uniform/normal draws (``sign``, ``u``, ``g``)
    so that the same particles can be regenerated for other parameters.
    """
    modes = [((m + 1) * k, a) for m, a in enumerate(alphas)]
    wl = two_stream(n_particles=n_particles, n_cells=n_cells, k=k, v_beam=v_beam,
                    v_spread=v_spread, dt=dt, steps=steps, order=order, seed=seed,
                    modes=modes)
    wl.name = "adjoint_two_stream"
    wl.meta.update(alphas=list(alphas), modes=modes)
    return wl


def catalogue() -> Dict[str, dict]:
    """The named full-size workloads, as keyword arguments of their builders."""
    return {
        "landau_1d1v_64c_100k": dict(builder="landau"),
        "two_stream_1d1v_512c_10M": dict(builder="two_stream"),
        # four times the particles: the 640 MB state no longer fits the Infinity Cache
        "two_stream_1d1v_512c_40M": dict(builder="two_stream", n_particles=40_000_000),
        "weibel_1d3v_256c_20M": dict(builder="weibel"),
        "batched_landau_512runs": dict(builder="batched_landau"),
        # one Landau run with the ensemble's total particle count (1.7 GB of state): the
        # plain passes at the batched form's size
        "landau_1d1v_512c_108M": dict(builder="landau", n_particles=107_838_210, n_cells=512),
        "adjoint_two_stream_256c_1M": dict(builder="adjoint_two_stream"),
    }


def by_name(name: str, **overrides):
    spec = dict(catalogue()[name])
    builder = globals()[spec.pop("builder")]
    spec.update(overrides)
    return builder(**spec)
