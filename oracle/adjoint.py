"""Test infrastructure (not part of the library): the discrete adjoint of the
oracle's RK4 trajectory, written plainly with the assembled operator, for
tiny meshes.

Objective (probe energy): J = sum_{n=1..N} dt sum_{T in probes} ||e^n||^2_{L2(T)},
with e^n the electric field after step n. In the oracle's Cartesian
coefficients with the orthonormal scalar basis, ||e||^2_{L2(T)} =
J_T sum_{c,l} c_{T,c,l}^2 (J_T = |det A_T|).

Gradient w.r.t. the per-element permittivity eps_T by the discrete adjoint of
classic RK4 (reverse sweep over the stages with the transposed operator):
every stage derivative is K_i = M^-1 (A X_i + b(t_i)); with the central flux
the stiffness A does not depend on eps, so dK_i/d eps_T at fixed X_i is
-(1/eps_T) times the E rows of K_i on element T. The time integrator is the
oracle's classic RK4 and the operator the oracle's (central flux, no PML).
Pinned by central finite differences of J (tests/test_oracle_adjoint.py).

With PML elements the state also carries the auxiliaries (p_E, p_H), in the
oracle's unscaled Cartesian form, which start at zero. Per Cartesian
component a of element T,
  d_t e = R_E / (eps J) - eta_a e - p_E / eps,   d_t p_E = -w_a p_E + eps xi_a e,
with R_E (curl, flux, current) free of eps for the central flux, so at fixed
state dF_E/deps_T = -(F_E + eta e)/eps_T and dF_pE/deps_T = xi e on the rows
of T, zero elsewhere. The adjoint sweep uses the transposed assembled
operator including the auxiliary rows.

Upwind flux: eps also enters the face weights through Z = sqrt(mu/eps), on
every face of T and in the neighbours' equations. There dF/deps_T at fixed
state is taken by central differences of the oracle's operator (relative
step 1e-5, on the rows of T and its neighbours, the only ones it touches);
the same route reproduces the analytic derivative above for the central
flux (pinned in tests/test_oracle_adjoint.py).
"""
import numpy as np


def probe_objective(O, cE0, cH0, dt, nsteps, probes):
    """J along the oracle's RK4 trajectory from (cE0, cH0) at t = 0 (PML
    auxiliaries, if any, from zero)."""
    pml = O.omega is not None
    s = [cE0, cH0, np.zeros_like(cE0) if pml else None, np.zeros_like(cH0) if pml else None]
    t = 0.0
    J = 0.0
    Jt = O.J[probes]
    for _ in range(nsteps):
        s = O.rk4_step(s, t, dt)
        t += dt
        J += dt * float(np.sum(Jt[:, None, None] * s[0][probes] ** 2))
    return J


def _assemble_with_aux(O):
    """Dense operator on (e, h, p_E, p_H) (no sources), for tiny meshes."""
    K, N, NH = O.K, O.N, O.NH
    sizes = [K * 3 * N, K * 3 * NH, K * 3 * N, K * 3 * NH]
    cuts = np.cumsum([0] + sizes)
    n = cuts[-1]
    Lm = np.zeros((n, n))
    dips = O.dipoles
    O.dipoles = []
    try:
        for col in range(n):
            v = np.zeros(n)
            v[col] = 1.0
            parts = [v[cuts[i]:cuts[i + 1]].reshape(K, 3, -1) for i in range(4)]
            d = O.rhs(*parts)
            Lm[:, col] = np.concatenate([x.ravel() for x in d])
    finally:
        O.dipoles = dips
    return Lm


def _with_eps(O, eps):
    """The same problem with another permittivity."""
    from .dg import OracleDG
    return OracleDG(O.verts, O.tets, O.p, eps=eps, mu=O.mu, flux=O.flux, omega=O.omega,
                    dipoles=[(pos, d, g) for (_, pos, d, g) in O.dipoles], ph=O.ph)


def adjoint_gradient(O, cE0, cH0, dt, nsteps, probes, deps=None):
    """(J, dJ/deps[K]) by the discrete adjoint of RK4 with the assembled operator.
    deps: "analytic" (central flux only) or "fd" (differences of the operator);
    default analytic for the central flux, fd for the upwind flux."""
    K, N = O.K, O.N
    nE = K * 3 * N
    pml = O.omega is not None
    deps = deps or ("analytic" if O.flux == "central" else "fd")
    if deps == "analytic" and O.flux != "central":
        raise ValueError("the analytic eps-derivative holds for the central flux only")
    if pml:
        from .dg import pml_tensors
        L = _assemble_with_aux(O)
        eta, xi = pml_tensors(O.omega)
        nEH = nE + K * 3 * O.NH
    else:
        L = O.assemble()  # no sources, E rows then H rows
    LT = L.T
    ntot = L.shape[0]

    def src(t):
        dE, dH, _, _ = O.rhs(np.zeros((K, 3, N)), np.zeros((K, 3, O.NH)), t=t, damping=False)
        v = np.zeros(ntot)
        v[:nE] = dE.ravel()
        v[nE:nE + dH.size] = dH.ravel()
        return v

    def F(x, t):
        return L @ x + src(t)

    # probe weights: d/dx of sum_T J_T |e_T|^2 is 2 W x (E rows of probes)
    w = np.zeros(ntot)
    for T in probes:
        w[T * 3 * N:(T + 1) * 3 * N] = O.J[T]
    x = [np.concatenate([cE0.ravel(), cH0.ravel(), np.zeros(ntot - nE - cH0.size)])]
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
    if deps == "fd":
        # per element: the perturbed problems, the element and its neighbours,
        # and their rows in the state vector (blocks e, h[, p_E, p_H])
        NH = O.NH
        blocks = [(0, N), (nE, NH)] + ([(nE + K * 3 * NH, N), (2 * nE + K * 3 * NH, NH)] if pml else [])
        fd = []
        for T in range(K):
            el = np.array([T] + [sd // 4 for sd in O.nbr_side[T] if sd >= 0], dtype=np.int64)
            rows = np.concatenate([off + (el[:, None] * 3 * nb + np.arange(3 * nb)[None, :]).ravel()
                                   for off, nb in blocks])
            h = 1e-5 * O.eps[T]
            ep, em = O.eps.copy(), O.eps.copy()
            ep[T] += h
            em[T] -= h
            fd.append((el, rows, h, _with_eps(O, ep), _with_eps(O, em)))

        def split(X):
            parts, off = [], 0
            for nb in (N, NH) + ((N, NH) if pml else ()):
                parts.append(X[off:off + K * 3 * nb].reshape(K, 3, nb))
                off += K * 3 * nb
            return parts + [None, None] * (not pml)

        def dF_rows(Op, X, t, el):
            d = Op.rhs(*split(X), t=t, elems=el)
            return np.concatenate([v.ravel() for v in d if v is not None])
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
        stages = ((kap1, k1, xn), (kap2, k2, xn + 0.5 * dt * k1), (kap3, k3, xn + 0.5 * dt * k2),
                  (kap4, k4, xn + dt * k3))
        if deps == "fd":
            for (kap, kk, X), ts in zip(stages, (t, t + 0.5 * dt, t + 0.5 * dt, t + dt)):
                for T, (el, rows, h, Op, Om) in enumerate(fd):
                    dF = (dF_rows(Op, X, ts, el) - dF_rows(Om, X, ts, el)) / (2.0 * h)
                    grad[T] += float(np.dot(kap[rows], dF))
            stages = ()
        for kap, kk, X in stages:
            dFE = kk[:nE]
            if pml:
                e = X[:nE].reshape(K, 3, N)
                dFE = dFE + (eta[:, :, None] * e).ravel()
                # p_E rows: dF/deps_T = xi e
                grad += np.bincount(erow, weights=kap[nEH:nEH + nE] * (xi[:, :, None] * e).ravel(), minlength=K)
            grad -= np.bincount(erow, weights=kap[:nE] * dFE, minlength=K) / O.eps
        lam = lam + mu1 + mu2 + mu3 + mu4
        if n >= 1:
            lam = lam + 2.0 * dt * w * xn
    return J, grad
