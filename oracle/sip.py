"""Symmetric interior penalty (SIP) surface unknown [KS Sec. III, eqs.
jmp_var_def, 1st_weak_equation, weak_penalty] on top of the oracle's central
operator, written plainly in physical Cartesian form (test infrastructure
only; see the package docstring).

System (central flux, PEC boundaries, optional PML and dipoles from OracleDG):

  (eps d_t e, v)_T = [central terms of OracleDG] - sum_F (h_s x n_T, v)_F
  (mu d_t h, w)_T  = [central terms of OracleDG]
  (mu_F/alpha_F) (d_t h_s, psi)_F = ([[e]]_F, psi)_F   for every face F

with h_s a tangential field on every face of the degree p_h of h (p with
equal orders; in the paper's mixed pairing, e at order p and h at p-1, it
is p-1). Readings (the paper leaves them open or garbled):

* jump: [[e]]_F = n_T x (e_T - e_T'), the same from either side T, T' of an
  interior face; on a PEC face [[e]]_F = n_T x e_T (the jump against the
  boundary value 0). These are the signs that make the paper's block system
  skew ((e, h, h_s) rows [0 C C_F; -C^T 0 0; -C_F^T 0 0]), so that
  W = 1/2 (eps e, e) + 1/2 (mu h, h) + 1/2 sum_F (mu_F/alpha_F) (h_s, h_s)_F
  is conserved (pinned in tests/test_oracle_sip.py).
* penalty: alpha_F = alpha0 (p+1)(p+3)/3 |F| / min(|T|, |T'|), p the order
  of e, whose jump is penalised (the trace inverse-inequality scaling of the
  cited lower bounds; one user constant alpha0 > 0); mu_F = (mu_T + mu_T')/2
  (mu_T on PEC faces).
* PML elements: h_s carries no damping (the penalty term is consistent, so
  it needs none).

Representation of h_s (the one the library's state arrays use, so that both
can be compared): face F with vertices a < b < c (ascending global id) is
parametrised as x = x_a + s1 (x_b - x_a) + s2 (x_c - x_a); h_s is stored by
its components along the edge tangents t1 = x_b - x_a, t2 = x_c - x_a,
    (h_s . t_k)(s) = sum_m S[F, k, m] psi_m(s1, s2),
with psi_m the orthonormal Dubiner basis of the parameter triangle (measure
ds1 ds2, written out in ``face_basis``). Here the tangential field of
coefficient (k, m) is built explicitly as the vector psi_m sum_l (g^-1)_kl t_l
(g_kl = t_k . t_l), and its face mass matrix is formed by quadrature.
"""
from __future__ import annotations

import math

import numpy as np

from .basis import jacobi, tri_quadrature
from .dg import FACE_VERTS
from .leapfrog import trapezoid_update


def face_modes(p):
    """(i, j) of the face basis: total degree d = i + j ascending, then i ascending."""
    return [(i, d - i) for d in range(p + 1) for i in range(d + 1)]


def face_basis(p, s):
    """Orthonormal Dubiner basis of P_p on the parameter triangle at s[..., 2]:
    psi_ij = sqrt(2 (2i+1)(i+j+1)) P_i^(0,0)(2 s2/(1-s1) - 1) (1-s1)^i
             P_j^(2i+1,0)(2 s1 - 1)   (points with s1 < 1)."""
    s = np.asarray(s, dtype=np.float64)
    s1, s2 = s[..., 0], s[..., 1]
    out = []
    for (i, j) in face_modes(p):
        a = jacobi(i, 0.0, 0.0, 2.0 * s2 / (1.0 - s1) - 1.0) * (1.0 - s1) ** i
        b = jacobi(j, 2.0 * i + 1.0, 0.0, 2.0 * s1 - 1.0)
        out.append(math.sqrt(2.0 * (2 * i + 1) * (i + j + 1)) * a * b)
    return np.stack(out, axis=-1)


class SipDG:
    """SIP extension of an OracleDG with the central flux (h_s of the order of h)."""

    def __init__(self, O, alpha0):
        if O.flux != "central":
            raise ValueError("SIP oracle: central flux")
        if not alpha0 > 0:
            raise ValueError("alpha0 > 0")
        self.O = O
        self.alpha0 = float(alpha0)
        p = O.p
        self.NF = (O.ph + 1) * (O.ph + 2) // 2  # face space of h_s: degree p_h
        K = O.K
        # unique faces, numbered by their first (element, face) side
        fid = -np.ones((K, 4), dtype=np.int64)
        sides = []
        for k in range(K):
            for f in range(4):
                if fid[k, f] >= 0:
                    continue
                fid[k, f] = len(sides)
                o = O.nbr_side[k, f]
                if o >= 0:
                    fid[o // 4, o % 4] = len(sides)
                sides.append((k, f, o))
        self.fid = fid
        self.sides = sides  # (element, local face, other side elem*4+face or -1)
        self.nfaces = len(sides)
        vol = O.J / 6.0
        self.fq, self.fw = tri_quadrature(p + 2)
        self.psi = face_basis(O.ph, self.fq)  # [Qf, NF]
        NF = self.NF
        self.alpha = np.zeros(self.nfaces)
        self.muF = np.zeros(self.nfaces)
        self.tang = np.zeros((self.nfaces, 2, 3))  # t1, t2
        self.vec = np.zeros((self.nfaces, 2, len(self.fw), NF, 3))  # tangential fields of (k, m)
        self.mass = np.zeros((self.nfaces, 2 * NF, 2 * NF))
        for F, (k, f, o) in enumerate(sides):
            xa, xb, xc = (O.X[k, v] for v in FACE_VERTS[f])
            t = np.stack([xb - xa, xc - xa])
            area = 0.5 * np.linalg.norm(np.cross(t[0], t[1]))
            vmin = vol[k] if o < 0 else min(vol[k], vol[o // 4])
            self.alpha[F] = self.alpha0 * (p + 1) * (p + 3) / 3.0 * area / vmin
            self.muF[F] = O.mu[k] if o < 0 else 0.5 * (O.mu[k] + O.mu[o // 4])
            self.tang[F] = t
            ginv = np.linalg.inv(t @ t.T)
            dual = ginv @ t  # rows: sum_l (g^-1)_kl t_l, so dual_k . t_j = delta_kj
            v = self.psi[None, :, :, None] * dual[:, None, None, :]  # [2, Qf, NF, 3]
            self.vec[F] = v
            w = self.fw * 2.0 * area  # physical weights (param triangle area 1/2)
            vv = v.transpose(1, 0, 2, 3).reshape(len(w), 2 * NF, 3)
            self.mass[F] = (self.muF[F] / self.alpha[F]) * np.einsum("q,qai,qbi->ab", w, vv, vv)

    # ---------------------------------------------------------- conversions
    def to_sides(self, S):
        """Per-face S[nfaces, 2, NF] -> per-side copies [K, 4, 2, NF]."""
        return S[self.fid]

    def from_sides(self, Ss):
        """Per-side copies [K, 4, 2, NF] -> per-face values (first side)."""
        return np.stack([Ss[k, f] for (k, f, _) in self.sides])

    def face_points(self, F):
        (k, f, _) = self.sides[F]
        xa = self.O.X[k, FACE_VERTS[f][0]]
        t = self.tang[F]
        return xa[None] + self.fq[:, :1] * t[0][None] + self.fq[:, 1:] * t[1][None]

    def hs_at(self, S, F):
        """h_s of face F at its quadrature points (tangential vectors) [Qf, 3]."""
        return np.einsum("km,kqmi->qi", S[F], self.vec[F])

    # ------------------------------------------------------------- operator
    def rhs(self, cE, cH, S, pE=None, pH=None, t=0.0, damping=True):
        """(dE, dH, dS, dpE, dpH): the oracle's central derivatives plus the
        h_s term of the E equation, and d_t h_s from the weak penalty equation."""
        O = self.O
        dE, dH, dpE, dpH = O.rhs(cE, cH, pE, pH, t=t, damping=damping)
        dE = dE.copy()
        dS = np.zeros_like(S)
        for F, (k, f, o) in enumerate(self.sides):
            x = self.face_points(F)
            area = 0.5 * np.linalg.norm(np.cross(self.tang[F][0], self.tang[F][1]))
            w = self.fw * 2.0 * area
            hs = self.hs_at(S, F)
            # E equation of every side T: -(h_s x n_T, phi_m e_i)_F / (eps_T J_T)
            sides = [(k, f)] + ([(o // 4, o % 4)] if o >= 0 else [])
            for (kk, ff) in sides:
                n = O.normal[kk, ff]
                r = O.Ainv[kk] @ (x - O.b[kk]).T
                phi = O.basis.eval(r.T)  # [Qf, N]
                FE = -np.cross(hs, n[None])
                dE[kk] += np.einsum("q,qi,qm->im", w, FE, phi) / (O.eps[kk] * O.J[kk])
            # weak penalty equation: M_F d_t S = ([[e]], psi)_F
            n = O.normal[k, f]
            em = O.eval_at(cE, np.full(len(w), k), x)
            ep = O.eval_at(cE, np.full(len(w), o // 4), x) if o >= 0 else np.zeros_like(em)
            jump = np.cross(n[None], em - ep)
            vv = self.vec[F].transpose(1, 0, 2, 3).reshape(len(w), 2 * self.NF, 3)
            rhs = np.einsum("q,qi,qai->a", w, jump, vv)
            dS[F] = np.linalg.solve(self.mass[F], rhs).reshape(2, self.NF)
        return dE, dH, dS, dpE, dpH

    def energy(self, cE, cH, S):
        """Field energy plus 1/2 sum_F (mu_F/alpha_F) (h_s, h_s)_F."""
        Ws = 0.5 * sum(float(s @ self.mass[F] @ s) for F, s in enumerate(S.reshape(self.nfaces, -1)))
        return self.O.energy(cE, cH) + Ws

    # ---------------------------------------------------------- time steps
    def rk4_run(self, cE, cH, S, pE=None, pH=None, t0=0.0, dt=1e-3, nsteps=1):
        """Classic RK4 on (e, h, h_s, p, q); returns ((e, h, h_s, p, q), t)."""
        O = self.O
        if O.omega is not None:
            pE = np.zeros_like(cE) if pE is None else pE
            pH = np.zeros_like(cH) if pH is None else pH
        s = [cE, cH, S, pE, pH]
        t = t0

        def L(u, tt):
            return list(self.rhs(u[0], u[1], u[2], u[3], u[4], t=tt))

        def axpy(u, k, a):
            return [None if x is None else x + a * y for x, y in zip(u, k)]

        for _ in range(nsteps):
            k1 = L(s, t)
            k2 = L(axpy(s, k1, 0.5 * dt), t + 0.5 * dt)
            k3 = L(axpy(s, k2, 0.5 * dt), t + 0.5 * dt)
            k4 = L(axpy(s, k3, dt), t + dt)
            s = [None if x is None else x + dt * (a / 6.0 + b / 3.0 + c / 3.0 + d / 6.0)
                 for x, a, b, c, d in zip(s, k1, k2, k3, k4)]
            t += dt
        return s, t

    def leapfrog_run(self, cE, cH, S, pE=None, pH=None, t0=0.0, dt=1e-3, nsteps=1):
        """The staggered scheme [KS Sec. V] with h_s beside h:
        e^{n+1} from (h, h_s)^{n+1/2} (sources at t + dt/2), then
        (h, h_s)^{n+3/2} from e^{n+1}; PML damping by the trapezoid rule."""
        O = self.O
        pml = O.omega is not None
        if pml:
            pE = np.zeros_like(cE) if pE is None else pE
            pH = np.zeros_like(cH) if pH is None else pH
        t = t0
        for _ in range(nsteps):
            kE, _, _, _, _ = self.rhs(cE, cH, S, t=t + 0.5 * dt, damping=False)
            if pml:
                cE, pE = trapezoid_update(O, cE, pE, kE, O.eps, dt)
            else:
                cE = cE + dt * kE
            _, kH, kS, _, _ = self.rhs(cE, cH, S, t=t + dt, damping=False)
            if pml:
                cH, pH = trapezoid_update(O, cH, pH, kH, O.mu, dt)
            else:
                cH = cH + dt * kH
            S = S + dt * kS
            t += dt
        return cE, cH, S, pE, pH, t

    def staggered_energy(self, cE, cH_prev, cH_next, S_prev, S_next):
        """1/2 (e, M_eps e) + 1/2 (h^-, M_mu h^+) + 1/2 (h_s^-, M_s h_s^+):
        conserved by the leap-frog scheme without sources and PML."""
        O = self.O
        J = O.J[:, None, None]
        We = 0.5 * float(np.sum(J * O.eps[:, None, None] * cE * cE))
        Wh = 0.5 * float(np.sum(J * O.mu[:, None, None] * cH_prev * cH_next))
        Ws = 0.5 * sum(float(a.ravel() @ self.mass[F] @ b.ravel()) for F, (a, b) in enumerate(zip(S_prev, S_next)))
        return We + Wh + Ws
