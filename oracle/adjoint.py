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
"""
import numpy as np


def probe_objective(O, cE0, cH0, dt, nsteps, probes):
    """J along the oracle's RK4 trajectory from (cE0, cH0) at t = 0."""
    s = [cE0, cH0, None, None]
    t = 0.0
    J = 0.0
    Jt = O.J[probes]
    for _ in range(nsteps):
        s = O.rk4_step(s, t, dt)
        t += dt
        J += dt * float(np.sum(Jt[:, None, None] * s[0][probes] ** 2))
    return J


def adjoint_gradient(O, cE0, cH0, dt, nsteps, probes):
    """(J, dJ/deps[K]) by the discrete adjoint of RK4 with the assembled operator."""
    K, N = O.K, O.N
    nE = K * 3 * N
    L = O.assemble()  # no sources, E rows then H rows
    LT = L.T

    def src(t):
        dE, dH, _, _ = O.rhs(np.zeros((K, 3, N)), np.zeros((K, 3, O.NH)), t=t)
        return np.concatenate([dE.ravel(), dH.ravel()])

    def F(x, t):
        return L @ x + src(t)

    # probe weights: d/dx of sum_T J_T |e_T|^2 is 2 W x (E rows of probes)
    w = np.zeros(nE + K * 3 * O.NH)
    for T in probes:
        w[T * 3 * N:(T + 1) * 3 * N] = O.J[T]
    x = [np.concatenate([cE0.ravel(), cH0.ravel()])]
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
        for kap, kk in ((kap1, k1), (kap2, k2), (kap3, k3), (kap4, k4)):
            grad -= np.bincount(erow, weights=kap[:nE] * kk[:nE], minlength=K) / O.eps
        lam = lam + mu1 + mu2 + mu3 + mu4
        if n >= 1:
            lam = lam + 2.0 * dt * w * xn
    return J, grad
