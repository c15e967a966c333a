"""Linear-theory reference values used by the physics pins (test helper, not a test).

Kinetic dispersion relations in the paper's units (omega_p = 1, lambda_D = 1,
q/m = +1), written with the plasma dispersion function Z(zeta) = i sqrt(pi) w(zeta)
(Faddeeva function from scipy).  These are textbook relations, independent of any code
in this repository.
"""
import math

import numpy as np
from scipy.optimize import fsolve
from scipy.special import wofz


def Z(z):
    return 1j * math.sqrt(math.pi) * wofz(z)


def _root(f, guess):
    def g(p):
        d = f(p[0] + 1j * p[1])
        return [d.real, d.imag]
    r = fsolve(g, [guess.real, guess.imag], xtol=1e-12)
    return r[0] + 1j * r[1]


def landau_root(k):
    """Least-damped root of 1 + (1 + zeta Z(zeta)) / k^2 = 0, zeta = omega / (sqrt(2) k)
    for a unit Maxwellian (section 5.1 quotes the approximate form of this rate)."""
    return _root(lambda w: 1 + (1 + (w / (k * math.sqrt(2))) * Z(w / (k * math.sqrt(2)))) / k ** 2,
                 complex(math.sqrt(1 + 3 * k * k), -0.1))


def landau_rate_paper_approx(k):
    """The approximate rate and Bohm-Gross frequency printed in section 5.1."""
    w2 = 1 + 3 * k * k
    return math.sqrt(math.pi / 2) * w2 / (2 * k ** 3) * math.exp(-w2 / (2 * k * k)), math.sqrt(w2)


def two_stream_cold_roots(k, vb, nb=0.5):
    """Roots of nb/(w - k vb)^2 + nb/(w + k vb)^2 = 1 (each beam has density nb)."""
    a = k * vb
    # nb[(w+a)^2 + (w-a)^2] = (w^2 - a^2)^2  ->  x^2 - (2a^2 + 2 nb) x + a^4 - 2 nb a^2 = 0
    b = 2 * a * a + 2 * nb
    c = a ** 4 - 2 * nb * a * a
    xs = np.roots([1.0, -b, c])
    return np.concatenate([np.sqrt(xs.astype(complex)), -np.sqrt(xs.astype(complex))])


def two_stream_warm_growth(k, vb, vt, nb=0.5):
    """Growth rate of two counter-streaming Maxwellian beams (density nb each, thermal
    speed vt): 1 + sum_b nb (1 + zeta_b Z(zeta_b)) / (k vt)^2 = 0,
    zeta_b = (omega - k v_b) / (sqrt(2) k vt)."""
    def D(w):
        s = 0
        for v in (vb, -vb):
            z = (w - k * v) / (math.sqrt(2) * k * vt)
            s += nb * (1 + z * Z(z)) / (k * vt) ** 2
        return 1 + s
    cold = max(two_stream_cold_roots(k, vb, nb), key=lambda w: w.imag)
    return _root(D, complex(0.0, cold.imag)).imag


def weibel_growth(k, vth_par, vth_perp, c=1.0):
    """Purely growing transverse mode for k along the cold (parallel) axis of a
    bi-Maxwellian: w^2 - c^2 k^2 - 1 + (T_perp/T_par) (1 + zeta Z(zeta)) = 0,
    zeta = w / (sqrt(2) k vth_par)."""
    A = (vth_perp / vth_par) ** 2

    def D(w):
        z = w / (math.sqrt(2) * k * vth_par)
        return w * w - c * c * k * k - 1 + A * (1 + z * Z(z))
    return _root(D, complex(0.0, 0.05)).imag


def mode_amplitude(field, m):
    """|Fourier coefficient m| of a periodic node array, scaled to the cosine amplitude."""
    return np.abs(np.fft.fft(field)[m]) * 2 / field.shape[-1]
