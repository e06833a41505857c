"""Plain FP64 DG Maxwell operator in physical Cartesian components (oracle).

Test infrastructure only (see the package docstring).

Semi-discrete system (paper Sec. III; fields e in P_pe(T)^3 and h in
P_ph(T)^3 on every tetrahedron T, Cartesian components, scalar basis
phi_m^T = phi_m o Phi_T^-1; equal orders by default, the paper's own choice
pe = ph + 1 with ph given, eqs. triale/trialh):

  E, weak curl with numerical flux (eq. uwc):
    (eps d_t e, v)_T = (h, curl v)_T - sum_F (h* x n, v)_F - (j, v)_T
  H, strong curl with consistent face term (eq. cwc):
    (mu d_t h, w)_T = -(curl e, w)_T + sum_F ((e* - e) x n, w)_F

n is the outward unit normal of T. Central flux (eq. uwc/cwc): h* and e* are
the arithmetic averages of the two traces. Upwind flux: the paper names
dissipative penalties without writing them (Sec. I); the reading used is the
exact Riemann solution of the 1-D impedance interface problem,
    n x h* = [n x (Z- h- + Z+ h+) - n x n x (e+ - e-)] / (Z- + Z+)
    n x e* = [n x (Y- e- + Y+ e+) + n x n x (h+ - h-)] / (Y- + Y+)
with Z = sqrt(mu/eps), Y = 1/Z.

PEC (Sec. IV, boundary of the truncated box): mirror ghost state on faces with
a single element, e+ = -e- + 2 n (n.e-), h+ = h-.

PML (Sec. IV, eqs. p_variable, q_variable, with per-axis damping w_a constant
per element): Laplace-domain stretching s_a = 1 + w_a/s gives
  s eps s_b s_c / s_a = eps (s + eta_a + xi_a/(s + w_a)),
  eta_a = w_b + w_c - w_a,  xi_a = (w_a - w_b)(w_a - w_c),
so, per Cartesian component a,
  eps d_t e_a + eps eta_a e_a + p_a = (curl terms)_a,   d_t p_a + w_a p_a = eps xi_a e_a
and the same for (h, q, mu). Each component uses its own pole w_a (exact
uniaxial layer); in face and corner regions this reduces to the paper's single
pole, and the eta/xi values reproduce the paper's listing (Appendix A).

Point current (j = d delta(r - r0) g(t), source term of eq. ampere_cont):
(j, v_m e_i)_T = g(t) d_i phi_m^T(r0) on the tet containing r0.

Time integration: classic four-stage Runge-Kutta.
"""
from __future__ import annotations

import numpy as np

from .basis import Dubiner, tet_quadrature, tri_quadrature

# local face f of a tet is opposite local vertex f; its vertices ascending
FACE_VERTS = ((1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2))

# (a x b)_i = eps_ijl a_j b_l
LEVI_CIVITA = np.zeros((3, 3, 3))
for _i, _j, _l in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
    LEVI_CIVITA[_i, _j, _l] = 1.0
    LEVI_CIVITA[_i, _l, _j] = -1.0


def pml_tensors(omega):
    """eta, xi (diagonal, per axis) of the per-component-pole PML, omega[...,3]."""
    w = np.asarray(omega, dtype=np.float64)
    wx, wy, wz = w[..., 0], w[..., 1], w[..., 2]
    eta = np.stack([wy + wz - wx, wz + wx - wy, wx + wy - wz], axis=-1)
    xi = np.stack([(wx - wy) * (wx - wz), (wy - wz) * (wy - wx), (wz - wx) * (wz - wy)], axis=-1)
    return eta, xi


class OracleDG:
    """Physical-space FP64 DG Maxwell operator on a tetrahedral mesh.

    Parameters
    ----------
    verts[nv,3], tets[nt,4] : mesh (any vertex order inside a tet).
    p : polynomial order of e (and of h unless ph is given).
    ph : polynomial order of h (default p); the paper pairs e at order ph+1
         with h at ph (eqs. triale, trialh). Test functions of each equation
         are those of its own field, so E and H coefficient arrays have
         N = dim P_p and NH = dim P_ph modes.
    eps, mu : per-element material (> 0).
    flux : "central" or "upwind".
    omega : [nt,3] per-axis PML damping (None = no PML).
    dipoles : list of (pos[3], dir[3], waveform callable g(t)).
    """

    def __init__(self, verts, tets, p, eps=None, mu=None, flux="central", omega=None,
                 dipoles=(), ph=None):
        self.verts = np.asarray(verts, dtype=np.float64)
        # canonical frame (only for the covariant conversions): ascending id
        self.tets = np.sort(np.asarray(tets, dtype=np.int64), axis=1)
        self.K = self.tets.shape[0]
        self.p = p
        self.ph = p if ph is None else int(ph)
        self.basis = Dubiner(p)  # e (and its test functions)
        self.N = self.basis.N
        self.basis_h = self.basis if self.ph == p else Dubiner(self.ph)  # h
        self.NH = self.basis_h.N
        self.eps = np.ones(self.K) if eps is None else np.asarray(eps, dtype=np.float64)
        self.mu = np.ones(self.K) if mu is None else np.asarray(mu, dtype=np.float64)
        if flux not in ("central", "upwind"):
            raise ValueError(flux)
        self.flux = flux
        self.omega = None if omega is None else np.asarray(omega, dtype=np.float64)
        X = self.verts[self.tets]  # [K,4,3]
        self.X = X
        self.b = X[:, 0].copy()
        self.A = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
        det = np.linalg.det(self.A)
        if not np.all(np.isfinite(det)) or np.any(np.abs(det) < 1e-300):
            raise ValueError("degenerate element")
        self.J = np.abs(det)
        self.Ainv = np.linalg.inv(self.A)
        self._faces()
        self.dipoles = []
        for (pos, d, g) in dipoles:
            k = self.locate(np.asarray(pos, dtype=np.float64))
            self.dipoles.append((k, np.asarray(pos, dtype=np.float64), np.asarray(d, dtype=np.float64), g))
        # every integrand is a product of two fields/test functions of degree
        # <= max(p, ph): rules exact to degree 2 max(p, ph) (2q - 1 >= that)
        q = max(p, self.ph) + 1
        self.vq, self.vw = tet_quadrature(q)
        self.fq, self.fw = tri_quadrature(q)
        self.phi_vq = self.basis.eval(self.vq)  # [Q, N]
        self.grad_vq = self.basis.grad(self.vq)  # [Q, 3, N]
        self.phih_vq = self.basis_h.eval(self.vq)  # [Q, NH]

    # ------------------------------------------------------------------ mesh
    def _faces(self):
        K = self.K
        keys = np.stack([self.tets[:, list(fv)] for fv in FACE_VERTS], axis=1).reshape(-1, 3)
        uniq, inv, cnt = np.unique(keys, axis=0, return_inverse=True, return_counts=True)
        inv = inv.ravel()
        if np.any(cnt > 2):
            raise ValueError("face shared by more than two elements")
        order = np.argsort(inv, kind="stable")
        nbr = -np.ones((K * 4,), dtype=np.int64)
        s = inv[order]
        pair = np.nonzero(s[1:] == s[:-1])[0]
        a, b = order[pair], order[pair + 1]
        nbr[a] = b
        nbr[b] = a
        self.nbr_side = nbr.reshape(K, 4)  # index k*4+f of the other side, or -1
        self.n_faces_interior = len(pair)
        self.n_faces_boundary = int(np.sum(cnt == 1))
        # physical outward unit normals and face vertex coordinates
        nrm = np.zeros((K, 4, 3))
        area2 = np.zeros((K, 4))
        for f, fv in enumerate(FACE_VERTS):
            xa, xb, xc = (self.X[:, v] for v in fv)
            c = np.cross(xb - xa, xc - xa)
            opp = self.X[:, f] - xa
            sgn = np.where(np.einsum("ij,ij->i", c, opp) > 0.0, -1.0, 1.0)
            a2 = np.linalg.norm(c, axis=1)
            nrm[:, f] = c * (sgn / a2)[:, None]
            area2[:, f] = a2
        self.normal = nrm
        self.area2 = area2  # |(xb-xa) x (xc-xa)| = 2 * area

    def locate(self, x):
        """Lowest-index element whose closed hull contains x (barycentric test)."""
        lam = np.einsum("kij,kj->ki", self.Ainv, x[None, :] - self.b)
        bary = np.concatenate([1.0 - lam.sum(axis=1, keepdims=True), lam], axis=1)
        inside = np.all(bary >= -1e-12, axis=1)
        idx = np.nonzero(inside)[0]
        if len(idx) == 0:
            raise ValueError("point outside mesh")
        return int(idx[0])

    # ----------------------------------------------------------- conversions
    def to_cartesian(self, u):
        """Covariant reference coefficients u[k,j,m] -> Cartesian c = A^-T u."""
        return np.einsum("kji,kjm->kim", self.Ainv, u)

    def to_covariant(self, c):
        """Cartesian coefficients c[k,i,m] -> covariant u = A^T c."""
        return np.einsum("kij,kim->kjm", self.A, c)

    def eval_at(self, coef, k, x):
        """Field of element(s) k at physical points x[...,3] -> [...,3]; the
        basis (of e or of h) follows the coefficient count."""
        r = np.einsum("...ij,...j->...i", self.Ainv[k], x - self.b[k])
        ph = (self.basis if coef.shape[2] == self.N else self.basis_h).eval(r)
        return np.einsum("...m,...im->...i", ph, coef[k])

    def project(self, fn, q=None, field="e"):
        """L2 projection of a physical vector field fn(x[...,3]) onto the space
        of e (c[K,3,N]) or, with field="h", of h (c[K,3,NH])."""
        q = self.p + 6 if q is None else q
        rq, w = tet_quadrature(q)
        ph = (self.basis if field == "e" else self.basis_h).eval(rq)  # [Q,N]
        x = self.b[:, None, :] + np.einsum("kij,qj->kqi", self.A, rq)  # [K,Q,3]
        F = fn(x)  # [K,Q,3]
        # (1/J) int_T F phi_m = sum_q w_q F(x_q) phi_m(r_q)
        return np.einsum("q,kqi,qm->kim", w, F, ph)

    # --------------------------------------------------------------- energy
    def energy(self, cE, cH):
        """W = 1/2 sum_T J_T (eps |c_E|^2 + mu |c_H|^2) (orthonormal scalar basis)."""
        return 0.5 * float(np.sum(self.J * (self.eps * np.sum(cE * cE, axis=(1, 2))
                                            + self.mu * np.sum(cH * cH, axis=(1, 2)))))

    # ---------------------------------------------------------------- flux
    def _flux(self, e_m, h_m, e_p, h_p, n, Zm, Zp):
        """Numerical fluxes (h*, e*) at face points (all arrays [...,3])."""
        if self.flux == "central":
            return 0.5 * (h_m + h_p), 0.5 * (e_m + e_p)
        Zm = Zm[..., None]
        Zp = Zp[..., None]
        Ym, Yp = 1.0 / Zm, 1.0 / Zp
        de = e_p - e_m
        dh = h_p - h_m
        # n x h* = [n x (Zm hm + Zp hp) - n x n x (e+ - e-)]/(Zm+Zp); only the
        # tangential part of h* enters (h* x n), so return a field whose
        # tangential part matches: h* = (Zm hm + Zp hp)/(ZS) - n x [e] / ZS
        hs = (Zm * h_m + Zp * h_p - np.cross(n, de)) / (Zm + Zp)
        # n x e* = [n x (Ym em + Yp ep) + n x n x (h+ - h-)]/(Ym+Yp)
        es = (Ym * e_m + Yp * e_p + np.cross(n, dh)) / (Ym + Yp)
        return hs, es

    # ------------------------------------------------------------------ rhs
    def rhs(self, cE, cH, pE=None, pH=None, t=0.0, elems=None, chunk=4096, damping=True):
        """Time derivatives (dcE, dcH, dpE, dpH) of the Cartesian coefficients.

        ``elems`` restricts the output to a subset of element indices (rows of
        the returned arrays follow ``elems``); the full state is still read for
        neighbours. pE/pH (PML auxiliaries, Cartesian, [K,3,N]) may be None.
        damping=False leaves out the PML terms (dpE = dpH = None): the
        undamped curl, flux and source terms only.
        """
        K, N, NH = self.K, self.N, self.NH
        idx_all = np.arange(K) if elems is None else np.asarray(elems, dtype=np.int64)
        # complex material values give the complex-step derivative by eps
        # (the operator is analytic in eps and mu)
        dtp = np.result_type(cE, cH, self.eps, self.mu)
        dE = np.zeros((len(idx_all), 3, N), dtype=dtp)
        dH = np.zeros((len(idx_all), 3, NH), dtype=dtp)
        Z = np.sqrt(self.mu / self.eps)
        for s in range(0, len(idx_all), chunk):
            idx = idx_all[s:s + chunk]
            RE, RH = self._rhs_chunk(cE, cH, idx, Z, t)
            dE[s:s + chunk] = RE / (self.eps[idx] * self.J[idx])[:, None, None]
            dH[s:s + chunk] = RH / (self.mu[idx] * self.J[idx])[:, None, None]
        dpE = dpH = None
        if self.omega is not None and damping:
            om = self.omega[idx_all]
            eta, xi = pml_tensors(om)
            pe = np.zeros((len(idx_all), 3, N)) if pE is None else pE[idx_all]
            ph = np.zeros((len(idx_all), 3, NH)) if pH is None else pH[idx_all]
            e = cE[idx_all]
            h = cH[idx_all]
            ep = self.eps[idx_all][:, None, None]
            mp = self.mu[idx_all][:, None, None]
            dE = dE - eta[:, :, None] * e - pe / ep
            dH = dH - eta[:, :, None] * h - ph / mp
            dpE = -om[:, :, None] * pe + ep * xi[:, :, None] * e
            dpH = -om[:, :, None] * ph + mp * xi[:, :, None] * h
        return dE, dH, dpE, dpH

    def _rhs_chunk(self, cE, cH, idx, Z, t):
        n = len(idx)
        N = self.N
        J = self.J[idx]
        AinvT = np.transpose(self.Ainv[idx], (0, 2, 1))  # grad phi = A^-T grad_hat
        # ---------------- volume terms (physical quadrature)
        G = np.einsum("kab,qbm->kqam", AinvT, self.grad_vq)  # [n,Q,3,N]
        phh = self.phih_vq  # [Q,NH]
        hq = np.einsum("kim,qm->kqi", cH[idx], phh)  # [n,Q,3]
        wJ = self.vw[None, :] * J[:, None]  # [n,Q]
        # E weak: (h, curl(phi_m e_i)) = e_i . (h x grad phi_m)
        RE = np.einsum("ijl,kqj,kqlm->kim", LEVI_CIVITA, wJ[:, :, None] * hq, G, optimize=True)
        # H strong: -(curl e, phi_m e_i), curl e = sum_n grad phi_n x c_n
        curl_e = np.einsum("ijl,kqjn,kln->kqi", LEVI_CIVITA, G, cE[idx], optimize=True)  # [n,Q,3]
        RH = -np.einsum("kqi,qm->kim", wJ[:, :, None] * curl_e, phh)
        RE = RE.astype(np.result_type(RE, Z))
        RH = RH.astype(np.result_type(RH, Z))
        # ---------------- face terms (physical face quadrature)
        s1 = self.fq[:, 0]
        s2 = self.fq[:, 1]
        for f, fv in enumerate(FACE_VERTS):
            xa = self.X[idx, fv[0]]
            xb = self.X[idx, fv[1]]
            xc = self.X[idx, fv[2]]
            x = xa[:, None] + s1[None, :, None] * (xb - xa)[:, None] + s2[None, :, None] * (xc - xa)[:, None]
            wq = self.fw[None, :] * self.area2[idx, f][:, None]  # [n,Qf]
            nrm = np.broadcast_to(self.normal[idx, f][:, None, :], x.shape)
            r_own = np.einsum("kij,kqj->kqi", self.Ainv[idx], x - self.b[idx][:, None])
            phi_own = self.basis.eval(r_own)
            phih_own = self.basis_h.eval(r_own)
            e_m = np.einsum("kqm,kim->kqi", phi_own, cE[idx])
            h_m = np.einsum("kqm,kim->kqi", phih_own, cH[idx])
            side = self.nbr_side[idx, f]
            has = side >= 0
            knb = np.where(has, side // 4, idx)
            # neighbour values at the same physical points via its inverse map
            r_nb = np.einsum("kij,kqj->kqi", self.Ainv[knb], x - self.b[knb][:, None])
            e_p = np.einsum("kqm,kim->kqi", self.basis.eval(r_nb), cE[knb])
            h_p = np.einsum("kqm,kim->kqi", self.basis_h.eval(r_nb), cH[knb])
            # PEC ghost
            en = np.sum(nrm * e_m, axis=-1, keepdims=True)
            e_ghost = -e_m + 2.0 * nrm * en
            e_p = np.where(has[:, None, None], e_p, e_ghost)
            h_p = np.where(has[:, None, None], h_p, h_m)
            Zm = np.broadcast_to(Z[idx][:, None], x.shape[:2])
            Zp = np.broadcast_to(Z[knb][:, None], x.shape[:2])
            hs, es = self._flux(e_m, h_m, e_p, h_p, nrm, Zm, Zp)
            FE = -np.cross(hs, nrm)
            FH = np.cross(es - e_m, nrm)
            RE += np.einsum("kqi,kqm->kim", wq[:, :, None] * FE, phi_own)
            RH += np.einsum("kqi,kqm->kim", wq[:, :, None] * FH, phih_own)
        # ---------------- point current source: -(j, phi_m e_i)
        for (k0, pos, d, g) in self.dipoles:
            sel = np.nonzero(idx == k0)[0]
            if len(sel):
                r = self.Ainv[k0] @ (pos - self.b[k0])
                phv = self.basis.eval(r[None, :])[0]
                RE[sel[0]] -= g(t) * np.outer(d, phv)
        return RE, RH

    # --------------------------------------------------------------- RK4
    def rk4_step(self, state, t, dt):
        """One classic RK4 step of (cE, cH, pE, pH) (pE/pH None without PML)."""
        def L(s, tt):
            dE, dH, dpE, dpH = self.rhs(s[0], s[1], s[2], s[3], tt)
            return [dE, dH, dpE, dpH]

        def axpy(s, k, a):
            return [None if x is None else x + a * y for x, y in zip(s, k)]

        k1 = L(state, t)
        k2 = L(axpy(state, k1, 0.5 * dt), t + 0.5 * dt)
        k3 = L(axpy(state, k2, 0.5 * dt), t + 0.5 * dt)
        k4 = L(axpy(state, k3, dt), t + dt)
        out = []
        for i, x in enumerate(state):
            if x is None:
                out.append(None)
            else:
                out.append(x + dt * (k1[i] / 6.0 + k2[i] / 3.0 + k3[i] / 3.0 + k4[i] / 6.0))
        return out

    def run(self, cE, cH, pE=None, pH=None, t0=0.0, dt=1e-3, nsteps=1):
        if self.omega is not None:
            pE = np.zeros_like(cE) if pE is None else pE
            pH = np.zeros_like(cH) if pH is None else pH
        s = [cE, cH, pE, pH]
        t = t0
        for _ in range(nsteps):
            s = self.rk4_step(s, t, dt)
            t += dt
        return s, t

    # -------------------------------------------------- dissipation identity
    def upwind_dissipation(self, cE, cH):
        """Energy rate of the upwind scheme, from an independent face loop.

        Interior faces (each once): -int_F |[e]_t|^2/(Z-+Z+) + |[h]_t|^2/(Y-+Y+) dS.
        PEC faces: only one element exists, so the mirror-ghost face carries half
        of that, -int_F |e_t|^2 / Z dS (derived from the 1-D Riemann flux)."""
        Z = np.sqrt(self.mu / self.eps)
        total = 0.0
        s1 = self.fq[:, 0]
        s2 = self.fq[:, 1]
        for k in range(self.K):
            for f, fv in enumerate(FACE_VERTS):
                side = self.nbr_side[k, f]
                if side >= 0 and side // 4 < k:
                    continue  # count interior faces once
                xa, xb, xc = (self.X[k, v] for v in fv)
                x = xa[None] + s1[:, None] * (xb - xa)[None] + s2[:, None] * (xc - xa)[None]
                n = self.normal[k, f]
                em = self.eval_at(cE, np.full(len(s1), k), x)
                hm = self.eval_at(cH, np.full(len(s1), k), x)
                if side >= 0:
                    kb = side // 4
                    ep = self.eval_at(cE, np.full(len(s1), kb), x)
                    hp = self.eval_at(cH, np.full(len(s1), kb), x)
                    Zp = Z[kb]
                else:
                    ep = -em + 2.0 * n[None] * (em @ n)[:, None]
                    hp = hm
                    Zp = Z[k]
                je = ep - em
                jh = hp - hm
                jet = je - np.outer(je @ n, n)
                jht = jh - np.outer(jh @ n, n)
                w = self.fw * self.area2[k, f]
                Zm = Z[k]
                half = 1.0 if side >= 0 else 0.5
                total -= half * np.sum(w * (np.sum(jet * jet, axis=1) / (Zm + Zp)
                                            + np.sum(jht * jht, axis=1) / (1.0 / Zm + 1.0 / Zp)))
        return total

    # ------------------------------------------------------ global operator
    def assemble(self):
        """Dense operator L (Cartesian, E then H, no PML/source) for tiny meshes."""
        K, N, NH = self.K, self.N, self.NH
        n = K * 3 * (N + NH)
        Lm = np.zeros((n, n))
        dips = self.dipoles
        self.dipoles = []
        try:
            for col in range(n):
                v = np.zeros(n)
                v[col] = 1.0
                cE = v[: K * 3 * N].reshape(K, 3, N)
                cH = v[K * 3 * N:].reshape(K, 3, NH)
                dE, dH, _, _ = self.rhs(cE, cH)
                Lm[:, col] = np.concatenate([dE.ravel(), dH.ravel()])
        finally:
            self.dipoles = dips
        return Lm

    def mass_diag(self):
        """Diagonal of the Cartesian mass matrix (E then H)."""
        K, N, NH = self.K, self.N, self.NH
        mE = np.repeat(self.eps * self.J, 3 * N)
        mH = np.repeat(self.mu * self.J, 3 * NH)
        return np.concatenate([mE, mH])
