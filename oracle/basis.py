"""Orthonormal modal basis on the reference tetrahedron and quadrature rules.

Oracle (test infrastructure only; see the package docstring).

Reference tetrahedron (Sec. II): T = {x,y,z >= 0, x+y+z <= 1}, vertices
(0,0,0), (1,0,0), (0,1,0), (0,0,1).

Basis (Sec. II, eq. dubiner_functions, ortho_cond). The printed formula is not
a polynomial basis as typeset: its middle factor lacks (1-x)^j and the last
Jacobi parameter should be (2i+2j+2, 0). The reading used here keeps the
paper's collapse roles (z innermost, then y, then x) and normalises to
L2(T)-orthonormality:

    phi_ijk = sqrt((2i+1)(2i+2j+2)(2i+2j+2k+3))
              * P_i^(0,0)(2z/(1-x-y) - 1) (1-x-y)^i
              * P_j^(2i+1,0)(2y/(1-x) - 1) (1-x)^j
              * P_k^(2i+2j+2,0)(2x - 1),          i+j+k <= p.

Mode order: total degree d = i+j+k ascending, then i ascending, then j
ascending.

Each basis function is expanded *exactly* into monomials x^a y^b z^c with
float64 coefficients, so values and gradients are plain polynomial
evaluations with no collapsed-coordinate singularities.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import polynomial as P1
from scipy.special import roots_jacobi


def modes(p: int):
    """Mode list [(i,j,k)] in the order described in the module docstring."""
    out = []
    for d in range(p + 1):
        for i in range(d + 1):
            for j in range(d - i + 1):
                out.append((i, j, d - i - j))
    return out


def jacobi_coeffs(n: int, a: float, b: float) -> np.ndarray:
    """Power-series coefficients (in w) of the Jacobi polynomial P_n^(a,b)(w).

    Three-term recurrence (Abramowitz & Stegun 22.7.1), with
    P_0 = 1 and P_1 = ((a-b) + (a+b+2) w) / 2.
    """
    p0 = np.array([1.0])
    if n == 0:
        return p0
    p1 = np.array([(a - b) / 2.0, (a + b + 2.0) / 2.0])
    for m in range(2, n + 1):
        c = 2.0 * m + a + b
        a1 = 2.0 * m * (m + a + b) * (c - 2.0)
        a2 = (c - 1.0) * (a * a - b * b)
        a3 = (c - 1.0) * c * (c - 2.0)
        a4 = 2.0 * (m + a - 1.0) * (m + b - 1.0) * c
        p2 = P1.polysub(P1.polyadd(a2 * p1, a3 * P1.polymulx(p1)), a4 * p0) / a1
        p0, p1 = p1, p2
    return p1


def jacobi(n: int, a: float, b: float, w) -> np.ndarray:
    """Evaluate P_n^(a,b)(w)."""
    return P1.polyval(np.asarray(w, dtype=np.float64), jacobi_coeffs(n, a, b))


class _Poly3:
    """Dense trivariate polynomial sum_{a,b,c} C[a,b,c] x^a y^b z^c."""

    def __init__(self, C):
        self.C = np.asarray(C, dtype=np.float64)

    @staticmethod
    def const(v, deg):
        C = np.zeros((deg + 1,) * 3)
        C[0, 0, 0] = v
        return _Poly3(C)

    @staticmethod
    def linear(c0, cx, cy, cz, deg):
        C = np.zeros((deg + 1,) * 3)
        C[0, 0, 0] = c0
        C[1, 0, 0] += cx
        C[0, 1, 0] += cy
        C[0, 0, 1] += cz
        return _Poly3(C)

    def __add__(self, o):
        return _Poly3(self.C + o.C)

    def scale(self, s):
        return _Poly3(self.C * s)

    def __mul__(self, o):
        d = self.C.shape[0] - 1
        out = np.zeros_like(self.C)
        nz = np.argwhere(self.C != 0.0)
        for (a, b, c) in nz:
            v = self.C[a, b, c]
            for (a2, b2, c2) in np.argwhere(o.C != 0.0):
                if a + a2 <= d and b + b2 <= d and c + c2 <= d:
                    out[a + a2, b + b2, c + c2] += v * o.C[a2, b2, c2]
        return _Poly3(out)

    def power(self, n):
        d = self.C.shape[0] - 1
        r = _Poly3.const(1.0, d)
        for _ in range(n):
            r = r * self
        return r

    def deriv(self, axis):
        d = self.C.shape[0] - 1
        out = np.zeros_like(self.C)
        for e in range(1, d + 1):
            src = [slice(None)] * 3
            dst = [slice(None)] * 3
            src[axis] = e
            dst[axis] = e - 1
            out[tuple(dst)] += e * self.C[tuple(src)]
        return _Poly3(out)


def _collapsed_factor(jc, lin_num, lin_den, deg):
    """sum_n jc[n] * lin_num^n * lin_den^(len(jc)-1-n), i.e.
    P(num/den) * den^order for a polynomial P of the given coefficients."""
    order = len(jc) - 1
    acc = _Poly3.const(0.0, deg)
    for n, cn in enumerate(jc):
        if cn == 0.0:
            continue
        acc = acc + (lin_num.power(n) * lin_den.power(order - n)).scale(cn)
    return acc


class Dubiner:
    """L2-orthonormal basis of P_p on the reference tetrahedron (monomial form)."""

    def __init__(self, p: int):
        self.p = p
        self.modes = modes(p)
        self.N = len(self.modes)
        deg = max(p, 1)  # construction degree (linear factors need >= 1)
        self.exps = [(a, b, c) for a in range(p + 1) for b in range(p + 1)
                     for c in range(p + 1) if a + b + c <= p]
        one_m_xy = _Poly3.linear(1.0, -1.0, -1.0, 0.0, deg)
        one_m_x = _Poly3.linear(1.0, -1.0, 0.0, 0.0, deg)
        # 2z/(1-x-y) - 1 = (2z - 1 + x + y)/(1-x-y)
        num_z = _Poly3.linear(-1.0, 1.0, 1.0, 2.0, deg)
        # 2y/(1-x) - 1 = (2y - 1 + x)/(1-x)
        num_y = _Poly3.linear(-1.0, 1.0, 2.0, 0.0, deg)
        w_x = _Poly3.linear(-1.0, 2.0, 0.0, 0.0, deg)
        unit = _Poly3.const(1.0, deg)
        polys = []
        for (i, j, k) in self.modes:
            f1 = _collapsed_factor(jacobi_coeffs(i, 0, 0), num_z, one_m_xy, deg)
            f2 = _collapsed_factor(jacobi_coeffs(j, 2 * i + 1, 0), num_y, one_m_x, deg)
            f3 = _collapsed_factor(jacobi_coeffs(k, 2 * i + 2 * j + 2, 0), w_x, unit, deg)
            nrm = math.sqrt((2 * i + 1) * (2 * i + 2 * j + 2) * (2 * i + 2 * j + 2 * k + 3))
            polys.append((f1 * f2 * f3).scale(nrm))
        self.polys = polys
        self.coef = np.array([[pl.C[e] for e in self.exps] for pl in polys])  # [N, nmon]
        self.dcoef = [np.array([[pl.deriv(ax).C[e] for e in self.exps] for pl in polys])
                      for ax in range(3)]

    def _monomials(self, pts):
        pts = np.asarray(pts, dtype=np.float64)
        x, y, z = pts[..., 0], pts[..., 1], pts[..., 2]
        d = max(self.p, 1)
        xp = [np.ones_like(x)]
        yp = [np.ones_like(y)]
        zp = [np.ones_like(z)]
        for _ in range(d):
            xp.append(xp[-1] * x)
            yp.append(yp[-1] * y)
            zp.append(zp[-1] * z)
        return np.stack([xp[a] * yp[b] * zp[c] for (a, b, c) in self.exps], axis=-1)

    def eval(self, pts):
        """Basis values at reference points pts[...,3] -> [..., N]."""
        return self._monomials(pts) @ self.coef.T

    def grad(self, pts):
        """Reference gradients -> [..., 3, N]."""
        m = self._monomials(pts)
        return np.stack([m @ dc.T for dc in self.dcoef], axis=-2)


def tet_quadrature(q: int):
    """Collapsed Gauss-Jacobi (conical product) rule on the reference tet.

    q points per direction, exact for total degree <= 2q-1. Weights sum to 1/6.
    """
    gx, wx = roots_jacobi(q, 2.0, 0.0)
    gy, wy = roots_jacobi(q, 1.0, 0.0)
    gz, wz = roots_jacobi(q, 0.0, 0.0)
    pts, w = [], []
    for a, wa in zip(gx, wx):
        x = 0.5 * (1.0 + a)
        for b, wb in zip(gy, wy):
            y = 0.5 * (1.0 + b) * (1.0 - x)
            for c, wc in zip(gz, wz):
                z = 0.5 * (1.0 + c) * (1.0 - x - y)
                pts.append((x, y, z))
                # dx dy dz = (1/2)(1/2)(1-x)(1/2)(1-x-y); (1-x)^2 and (1-y')
                # factors are absorbed by the Jacobi weights
                w.append(wa * wb * wc / 64.0)
    return np.array(pts), np.array(w)


def tri_quadrature(q: int):
    """Collapsed rule on the parameter triangle {s1,s2 >= 0, s1+s2 <= 1}.

    Exact for total degree <= 2q-1; weights sum to 1/2.
    """
    ga, wa = roots_jacobi(q, 1.0, 0.0)
    gb, wb = roots_jacobi(q, 0.0, 0.0)
    pts, w = [], []
    for a, w1 in zip(ga, wa):
        s1 = 0.5 * (1.0 + a)
        for b, w2 in zip(gb, wb):
            s2 = 0.5 * (1.0 + b) * (1.0 - s1)
            pts.append((s1, s2))
            w.append(w1 * w2 / 8.0)
    return np.array(pts), np.array(w)
