"""50-digit brute-force reference of one particle-in-cell step, for a handful of particles.

TEST INFRASTRUCTURE ONLY (part of the oracle).  Written independently of
``pic_oracle.c`` and deliberately structured differently, so that the two agreeing says
more than either alone:

* the shape function is evaluated at *every* node against every periodic image of the
  particle, ``S(x_i - x_p + m L)`` for ``m = -1, 0, 1`` (section 2.2, the tent
  ``max(0, 1 - |z|/h)`` and the degree-2 B-spline written as a convolution of the tent
  with a unit box, see ``_bspline2``);
* the Crank-Nicolson field system of eq. (EMbasic) is assembled as a dense matrix from
  the difference operators and solved by Gaussian elimination (``mpmath.lu_solve``);
* the half-step velocity of eq. (good_translation)/(EMbasic) is found by solving the
  3x3 linear system ``v - (dt/2) v x B = u`` directly, not by a closed form.

Steps follow eq. (good_translation) (ESEC2), eq. (naivetranslation) with
eq. (PICmodification) (ESEC1) and eq. (EMbasic) (EMEC(LI)); the correction is
eq. (opt_solution) with the fallback Gamma := 1 when the radicand is negative
(section 3.2).  Energies follow section 5.1.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import mpmath as mp

mp.mp.dps = 50


def _tent(t):
    t = abs(t)
    return 1 - t if t < 1 else mp.mpf(0)


def _bspline2(t):
    """Degree-2 B-spline as the convolution of the tent with the unit box on
    [-1/2, 1/2]: the integral of the tent over [t - 1/2, t + 1/2], done exactly on the
    tent's two linear pieces."""
    def tent_integral(a, b):       # integral of max(0, 1 - |s|) over [a, b]
        def F(s):                  # antiderivative, clamped to the support [-1, 1]
            s = min(max(s, mp.mpf(-1)), mp.mpf(1))
            return s + s * abs(s) / 2 * (-1)
        return F(b) - F(a)
    return tent_integral(t - mp.mpf(1) / 2, t + mp.mpf(1) / 2)


def shape(order: int, t):
    return _tent(t) if order == 1 else _bspline2(t)


def _S(order, xnode, xp, h, L):
    """Periodic shape: the sum over images of S(x_node - x_p + m L).  The sum is
    L-periodic in x_p, so x_p is first reduced into [0, L); then the images
    m = -1, 0, 1 cover every node within the support (at most 3h/2 < L)."""
    xp = xp - L * mp.floor(xp / L)
    return sum(shape(order, (xnode - xp + m * L) / h) for m in (-1, 0, 1))


def deposit(order, xs, q, ng, h, L, shift=0):
    out = [mp.mpf(0)] * ng
    for i in range(ng):
        xi = (i + mp.mpf(shift)) * h
        out[i] = sum(qp * _S(order, xi, xp, h, L) for xp, qp in zip(xs, q)) / h
    return out


def gather(order, xs, field, h, L, shift=0):
    ng = len(field)
    return [sum(field[i] * _S(order, (i + mp.mpf(shift)) * h, xp, h, L) for i in range(ng))
            for xp in xs]


def _cross(a, b):
    return [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]


def _solve_half_velocity(u, t):
    """v with v = u + v x t, by solving the 3x3 system (I - [x t]) v = u."""
    # (v x t)_r = sum_c M[r][c] v_c with M = [[0, t2, -t1], [-t2, 0, t0], [t1, -t0, 0]]
    M = mp.matrix([[1, -t[2], t[1]], [t[2], 1, -t[0]], [-t[1], t[0], 1]])
    sol = mp.lu_solve(M, mp.matrix(u))
    return [sol[0], sol[1], sol[2]]


class MPState:
    """Tiny periodic 1D system held in 50-digit numbers.

    ``x``: positions; ``v``: list of nv lists; ``w``: weights; ``E``: 3 node arrays (only
    E_x used electrostatically); ``B``: (B_y, B_z) on the half nodes."""

    def __init__(self, nv, scheme, order, ng, L, dt, x, v, w, E, B=None, c=1.0,
                 b_ext=(0, 0, 0)):
        self.nv, self.scheme, self.order, self.ng = nv, scheme, order, ng
        self.L, self.dt, self.c = mp.mpf(L), mp.mpf(dt), mp.mpf(c)
        self.h = self.L / ng
        self.x = [mp.mpf(a) for a in x]
        self.v = [[mp.mpf(a) for a in comp] for comp in v]
        self.w = [mp.mpf(a) for a in w]
        self.E = [[mp.mpf(a) for a in comp] for comp in E]
        self.B = [[mp.mpf(a) for a in comp] for comp in (B if B is not None else [[0] * ng] * 2)]
        self.bext = [mp.mpf(a) for a in b_ext]
        self.fallbacks = 0
        self.gammas: List = []

    # ---------------------------------------------------------------- energies
    def energy(self):
        ke = sum(wp * sum(self.v[c][p] ** 2 for c in range(self.nv)) / 2
                 for p, wp in enumerate(self.w))
        ne = 3 if self.scheme == "emec_li" else 1
        we = self.h / 2 * sum(self.E[c][i] ** 2 for c in range(ne) for i in range(self.ng))
        wb = mp.mpf(0)
        if self.scheme == "emec_li":
            wb = self.c ** 2 * self.h / 2 * sum(b ** 2 for comp in self.B for b in comp)
        return ke, we, wb, ke + we + wb

    # ------------------------------------------------------------- operators
    def _dplus(self, f):      # nodes -> half nodes
        return [(f[(i + 1) % self.ng] - f[i]) / self.h for i in range(self.ng)]

    def _dminus(self, g):     # half nodes -> nodes
        return [(g[i] - g[i - 1]) / self.h for i in range(self.ng)]

    def _cn_matrix(self, s):
        n, h = self.ng, self.h
        A = mp.zeros(n, n)
        for i in range(n):
            A[i, i] += 1 + 2 * s / h ** 2
            A[i, (i + 1) % n] += -s / h ** 2
            A[i, (i - 1) % n] += -s / h ** 2
        return A

    def _lap(self, f):
        n, h = self.ng, self.h
        return [(f[(i + 1) % n] - 2 * f[i] + f[(i - 1) % n]) / h ** 2 for i in range(n)]

    # ------------------------------------------------------------------ step
    def step(self):
        nv, ng, h, L, dt, o = self.nv, self.ng, self.h, self.L, self.dt, self.order
        em = self.scheme == "emec_li"
        npart = len(self.x)
        half = dt / 2
        xs = [self.x[p] + half * self.v[0][p] for p in range(npart)]
        ncur = 3 if em else 1
        # predictor fields
        if self.scheme == "esec1":
            Es = [list(self.E[0]), [0] * ng, [0] * ng]
            Bs = self.B
        else:
            J1 = [deposit(o, xs, [self.w[p] * self.v[c][p] for p in range(npart)], ng, h, L)
                  for c in range(ncur)]
            if not em:
                m = sum(J1[0]) / ng
                Es = [[self.E[0][i] - half * (J1[0][i] - m) for i in range(ng)],
                      [0] * ng, [0] * ng]
                Bs = self.B
            else:
                c2 = self.c ** 2
                dBy, dBz = self._dminus(self.B[0]), self._dminus(self.B[1])
                Es = [[self.E[0][i] - half * J1[0][i] for i in range(ng)],
                      [self.E[1][i] + half * (-c2 * dBz[i] - J1[1][i]) for i in range(ng)],
                      [self.E[2][i] + half * (c2 * dBy[i] - J1[2][i]) for i in range(ng)]]
                dEz, dEy = self._dplus(self.E[2]), self._dplus(self.E[1])
                Bs = [[self.B[0][i] + half * dEz[i] for i in range(ng)],
                      [self.B[1][i] - half * dEy[i] for i in range(ng)]]
        ne = 3 if em else 1
        gE = [gather(o, xs, Es[c], h, L) for c in range(ne)]
        vs = [[None] * npart for _ in range(nv)]
        for p in range(npart):
            if nv == 1:
                vs[0][p] = self.v[0][p] + half * gE[0][p]
            else:
                B = list(self.bext)
                if em:
                    B[1] += gather(o, [xs[p]], Bs[0], h, L, shift=0.5)[0]
                    B[2] += gather(o, [xs[p]], Bs[1], h, L, shift=0.5)[0]
                u = [self.v[c][p] + half * (gE[c][p] if c < ne else 0) for c in range(3)]
                sol = _solve_half_velocity(u, [half * b for b in B])
                for c in range(3):
                    vs[c][p] = sol[c]
        x1 = [self.x[p] + dt * vs[0][p] for p in range(npart)]
        xh = [(self.x[p] + x1[p]) / 2 for p in range(npart)]
        J2 = [deposit(o, xh, [self.w[p] * vs[c][p] for p in range(npart)], ng, h, L)
              for c in range(ncur)]
        if not em:
            m = sum(J2[0]) / ng
            En = [[self.E[0][i] - dt * (J2[0][i] - m) for i in range(ng)], [0] * ng, [0] * ng]
            Bn = self.B
        else:
            c2 = self.c ** 2
            s = half ** 2 * c2
            A = self._cn_matrix(s)
            lapy, lapz = self._lap(self.E[1]), self._lap(self.E[2])
            dBy, dBz = self._dminus(self.B[0]), self._dminus(self.B[1])
            ry = [self.E[1][i] + s * lapy[i] - dt * c2 * dBz[i] - dt * J2[1][i] for i in range(ng)]
            rz = [self.E[2][i] + s * lapz[i] + dt * c2 * dBy[i] - dt * J2[2][i] for i in range(ng)]
            Ey = mp.lu_solve(A, mp.matrix(ry))
            Ez = mp.lu_solve(A, mp.matrix(rz))
            En = [[self.E[0][i] - dt * J2[0][i] for i in range(ng)],
                  [Ey[i] for i in range(ng)], [Ez[i] for i in range(ng)]]
            sy = self._dplus([self.E[1][i] + En[1][i] for i in range(ng)])
            sz = self._dplus([self.E[2][i] + En[2][i] for i in range(ng)])
            Bn = [[self.B[0][i] + half * sz[i] for i in range(ng)],
                  [self.B[1][i] - half * sy[i] for i in range(ng)]]
        Eb = [[(self.E[c][i] + En[c][i]) / 2 for i in range(ng)] for c in range(3)]
        Bb = [[(self.B[c][i] + Bn[c][i]) / 2 for i in range(ng)] for c in range(2)]
        gEb = [gather(o, xh, Eb[c], h, L) for c in range(ne)]
        newv = [[None] * npart for _ in range(nv)]
        self.gammas = []
        for p in range(npart):
            vn = [self.v[c][p] for c in range(nv)]
            vstar = [vs[c][p] for c in range(nv)]
            if nv == 1:
                vd = [vn[0] + dt * gEb[0][p]]
            else:
                B = list(self.bext)
                if em:
                    B[1] += gather(o, [xh[p]], Bb[0], h, L, shift=0.5)[0]
                    B[2] += gather(o, [xh[p]], Bb[1], h, L, shift=0.5)[0]
                vxb = _cross(vstar, B)
                vd = [vn[c] + dt * ((gEb[c][p] if c < ne else 0) + vxb[c]) for c in range(3)]
            num = sum((vstar[c] - (vd[c] + vn[c]) / 2) * (vd[c] - vn[c]) for c in range(nv))
            den = sum(a * a for a in vd)
            r = 1 + 2 * num / den
            if r >= 0:
                g = mp.sqrt(r)
            else:
                g = mp.mpf(1)
                self.fallbacks += 1
            self.gammas.append(g)
            for c in range(nv):
                newv[c][p] = g * vd[c]
        self.v = newv
        self.x = [a - L * mp.floor(a / L) for a in x1]
        self.E = [list(En[c]) if c < (3 if em else 1) else self.E[c] for c in range(3)]
        if em:
            self.B = [list(Bn[0]), list(Bn[1])]


def run(nv, scheme, order, ng, L, dt, x, v, w, E, B=None, c=1.0, b_ext=(0, 0, 0),
        steps=1) -> MPState:
    st = MPState(nv, scheme, order, ng, L, dt, x, v, w, E, B, c, b_ext)
    for _ in range(steps):
        st.step()
    return st
