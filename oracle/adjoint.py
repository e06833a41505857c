"""Test infrastructure (not part of the library): the discrete adjoint of the
oracle's RK4 trajectory, written plainly with the assembled operator, for
tiny meshes.

Objective (probe energy): J = sum_{n=1..N} dt sum_{T in probes} ||e^n||^2_{L2(T)},
with e^n the electric field after step n. In the oracle's Cartesian
coefficients with the orthonormal scalar basis, ||e||^2_{L2(T)} =
J_T sum_{c,l} c_{T,c,l}^2 (J_T = |det A_T|).

Gradient w.r.t. the per-element permittivity eps_T by the discrete adjoint of
classic RK4 (reverse sweep over the stages with the transposed operator):
every stage derivative is K_i = F(X_i, t_i) = L X_i + b(t_i), and
dJ/deps_T = sum over steps and stages of (kappa_i, dF/deps_T (X_i, t_i)),
kappa_i the adjoint stage weights.

State vector: (e, h[, h_s][, p_E, p_H]) in the oracle's Cartesian
coefficients; h_s (the SIP surface unknown of [KS Sec. III], per face, see
``sip.py``) and the PML auxiliaries (unscaled, [KS Sec. IV]) start at zero.

How eps enters F at fixed state (eps_T only acts on the rows of T and, with
the upwind flux, of its face neighbours):
* central flux, with or without PML or h_s: the curl, flux, h_s and current
  terms of the E equation are divided by eps_T and nothing else in them
  depends on eps; per Cartesian component a of a PML element
      d_t e = R_E / (eps J) - eta_a e - p_E / eps,  d_t p_E = -w_a p_E + eps xi_a e,
  so dF_E/deps_T = -(F_E + eta e)/eps_T and dF_pE/deps_T = xi e on the rows
  of T (the h_s rows do not involve eps: their face mass holds mu_F and
  alpha_F only);
* upwind flux: eps also enters the face weights through Z = sqrt(mu/eps), on
  every face of T and in the neighbours' equations. There dF/deps_T is taken
  by complex-step differentiation of the oracle's operator, which is an
  analytic function of eps: dF/deps_T = Im F(eps + i delta e_T) / delta with
  delta = 1e-20 eps_T, exact to rounding (no difference of two values is
  formed). The same route reproduces the closed form of the central flux
  (pinned in tests/test_oracle_adjoint.py).
"""
import copy

import numpy as np


def probe_objective(O, cE0, cH0, dt, nsteps, probes, sip=None):
    """J along the oracle's RK4 trajectory from (cE0, cH0) at t = 0 (PML
    auxiliaries and, with ``sip`` (a SipDG on O), h_s from zero)."""
    pml = O.omega is not None
    Jt = O.J[probes]
    if sip is not None:
        S = np.zeros((sip.nfaces, 2, sip.NF))
        J = 0.0
        s = (cE0, cH0, S, None, None)
        for n in range(nsteps):
            s, _ = sip.rk4_run(*s, t0=n * dt, dt=dt, nsteps=1)
            J += dt * float(np.sum(Jt[:, None, None] * s[0][probes] ** 2))
        return J
    s = [cE0, cH0, np.zeros_like(cE0) if pml else None, np.zeros_like(cH0) if pml else None]
    t = 0.0
    J = 0.0
    for _ in range(nsteps):
        s = O.rk4_step(s, t, dt)
        t += dt
        J += dt * float(np.sum(Jt[:, None, None] * s[0][probes] ** 2))
    return J


class _Layout:
    """Blocks of the state vector: e, h, [h_s], [p_E, p_H]."""

    def __init__(self, O, sip):
        K = O.K
        self.pml = O.omega is not None
        self.sip = sip
        self.shapes = [("e", (K, 3, O.N)), ("h", (K, 3, O.NH))]
        if sip is not None:
            self.shapes.append(("s", (sip.nfaces, 2, sip.NF)))
        if self.pml:
            self.shapes += [("pE", (K, 3, O.N)), ("pH", (K, 3, O.NH))]
        self.off = {}
        o = 0
        for name, shp in self.shapes:
            self.off[name] = o
            o += int(np.prod(shp))
        self.n = o

    def split(self, v):
        d = {name: v[self.off[name]:self.off[name] + int(np.prod(shp))].reshape(shp) for name, shp in self.shapes}
        return d

    def rhs(self, Op, v, t=0.0, elems=None, damping=True):
        """Derivative of the state vector v by the operator of Op (an
        OracleDG, or with h_s its SipDG), as a vector; with elems only the
        element rows of e, h, p_E, p_H of those elements (in the order of
        ``element_rows``)."""
        d = self.split(v)
        if self.sip is not None:
            dE, dH, dS, dpE, dpH = Op.rhs(d["e"], d["h"], d["s"], d.get("pE"), d.get("pH"), t=t, damping=damping)
            parts = [dE, dH, dS]
        else:
            dE, dH, dpE, dpH = Op.rhs(d["e"], d["h"], d.get("pE"), d.get("pH"), t=t, elems=elems, damping=damping)
            parts = [dE, dH]
        if self.pml:  # without damping the auxiliaries have no derivative
            parts += [np.zeros_like(dE) if dpE is None else dpE, np.zeros_like(dH) if dpH is None else dpH]
        return np.concatenate([x.ravel() for x in parts])

    def element_rows(self, O, el):
        """Rows of the element blocks (e, h, p_E, p_H) of elements el, in the
        order rhs(elems=el) returns them."""
        rows = []
        for name, shp in self.shapes:
            if name == "s":
                continue
            nb = shp[1] * shp[2]
            rows.append(self.off[name] + (el[:, None] * nb + np.arange(nb)[None, :]).ravel())
        return np.concatenate(rows)


def assemble(O, sip=None):
    """Dense operator on the state vector (e, h[, h_s][, p_E, p_H]) without
    sources, one column per unit vector, for tiny meshes."""
    lay = _Layout(O, sip)
    Op = sip if sip is not None else O
    dips = O.dipoles
    O.dipoles = []
    try:
        Lm = np.zeros((lay.n, lay.n))
        for col in range(lay.n):
            v = np.zeros(lay.n)
            v[col] = 1.0
            Lm[:, col] = lay.rhs(Op, v)
    finally:
        O.dipoles = dips
    return Lm


def _with_complex_eps(O, T, delta):
    """A shallow copy of O whose permittivity is eps + i delta on element T."""
    Oc = copy.copy(O)
    eps = O.eps.astype(np.complex128)
    eps[T] += 1j * delta
    Oc.eps = eps
    return Oc


def adjoint_gradient(O, cE0, cH0, dt, nsteps, probes, deps=None, sip=None):
    """(J, dJ/deps[K]) by the discrete adjoint of RK4 with the assembled operator.
    deps: "analytic" (central flux only) or "complex" (complex-step
    derivative of the operator on the rows of each element and its
    neighbours); default analytic for the central flux, complex for the
    upwind flux. sip: a SipDG on O (central flux) to carry the surface
    unknown h_s (from zero)."""
    K, N = O.K, O.N
    lay = _Layout(O, sip)
    pml = lay.pml
    deps = deps or ("analytic" if O.flux == "central" else "complex")
    if deps == "analytic" and O.flux != "central":
        raise ValueError("the analytic eps-derivative holds for the central flux only")
    L = assemble(O, sip)
    LT = L.T
    ntot = lay.n
    nE = K * 3 * N
    if pml:
        from .dg import pml_tensors
        eta, xi = pml_tensors(O.omega)
    Op = sip if sip is not None else O

    def src(t):
        return lay.rhs(Op, np.zeros(ntot), t=t, damping=False)

    def F(x, t):
        return L @ x + src(t)

    # probe weights: d/dx of sum_T J_T |e_T|^2 is 2 W x (E rows of probes)
    w = np.zeros(ntot)
    for T in probes:
        w[T * 3 * N:(T + 1) * 3 * N] = O.J[T]
    x = [np.zeros(ntot)]
    x[0][:nE] = cE0.ravel()
    x[0][lay.off["h"]:lay.off["h"] + cH0.size] = cH0.ravel()
    J = 0.0
    for n in range(nsteps):
        t = n * dt
        xn = x[-1]
        k1 = F(xn, t)
        k2 = F(xn + 0.5 * dt * k1, t + 0.5 * dt)
        k3 = F(xn + 0.5 * dt * k2, t + 0.5 * dt)
        k4 = F(xn + dt * k3, t + dt)
        x.append(xn + dt * (k1 / 6.0 + k2 / 3.0 + k3 / 3.0 + k4 / 6.0))
        J += dt * float(np.sum(w * x[-1] ** 2))
    grad = np.zeros(K)
    lam = 2.0 * dt * w * x[nsteps]
    erow = np.repeat(np.arange(K), 3 * N)  # element of each E row
    if deps == "complex":
        # per element: the complex-eps problem, the element and its
        # neighbours, and their rows in the state vector
        cs = []
        for T in range(K):
            el = np.array([T] + [sd // 4 for sd in O.nbr_side[T] if sd >= 0], dtype=np.int64)
            delta = 1e-20 * O.eps[T]
            Oc = _with_complex_eps(O, T, delta)
            if sip is not None:  # the same surface unknown on the complex-eps operator
                Oc_sip = copy.copy(sip)
                Oc_sip.O = Oc
                Oc = Oc_sip
            cs.append((el, lay.element_rows(O, el), delta, Oc))
    for n in range(nsteps - 1, -1, -1):
        t = n * dt
        xn = x[n]
        k1 = F(xn, t)
        k2 = F(xn + 0.5 * dt * k1, t + 0.5 * dt)
        k3 = F(xn + 0.5 * dt * k2, t + 0.5 * dt)
        k4 = F(xn + dt * k3, t + dt)
        kap4 = dt / 6.0 * lam
        mu4 = LT @ kap4
        kap3 = dt / 3.0 * lam + dt * mu4
        mu3 = LT @ kap3
        kap2 = dt / 3.0 * lam + 0.5 * dt * mu3
        mu2 = LT @ kap2
        kap1 = dt / 6.0 * lam + 0.5 * dt * mu2
        mu1 = LT @ kap1
        stages = ((kap1, k1, xn, t), (kap2, k2, xn + 0.5 * dt * k1, t + 0.5 * dt),
                  (kap3, k3, xn + 0.5 * dt * k2, t + 0.5 * dt), (kap4, k4, xn + dt * k3, t + dt))
        for kap, kk, X, ts in stages:
            if deps == "complex":
                for T, (el, rows, delta, Oc) in enumerate(cs):
                    if sip is not None:  # the h_s rows do not involve eps
                        dF = lay.rhs(Oc, X, t=ts)[rows].imag / delta
                    else:
                        dF = lay.rhs(Oc, X, t=ts, elems=el).imag / delta
                    grad[T] += float(np.dot(kap[rows], dF))
                continue
            dFE = kk[:nE]
            if pml:
                e = X[:nE].reshape(K, 3, N)
                dFE = dFE + (eta[:, :, None] * e).ravel()
                # p_E rows: dF/deps_T = xi e
                pE0 = lay.off["pE"]
                grad += np.bincount(erow, weights=kap[pE0:pE0 + nE] * (xi[:, :, None] * e).ravel(), minlength=K)
            grad -= np.bincount(erow, weights=kap[:nE] * dFE, minlength=K) / O.eps
        lam = lam + mu1 + mu2 + mu3 + mu4
        if n >= 1:
            lam = lam + 2.0 * dt * w * xn
    return J, grad
