"""Test infrastructure: the staggered leap-frog time scheme the paper uses for
its experiments [KS Sec. V] with the oracle's operator, written plainly.

State (e^n, h^{n+1/2}). With the central flux the E derivative depends only
on h (and the current j) and the H derivative only on e, so one step is
    e^{n+1}   = e^n       + dt dE(h^{n+1/2}, t^{n+1/2})
    h^{n+3/2} = h^{n+1/2} + dt dH(e^{n+1})
The quantity W^n = 1/2 (e^n, M_eps e^n) + 1/2 (h^{n-1/2}, M_mu h^{n+1/2}) is
conserved exactly without sources (pinned in tests/test_oracle_leapfrog.py).
Equal orders for e and h. With PML elements the damping terms are taken by
the trapezoid rule (leapfrog_pml_step, pinned by second-order convergence to
the RK4-resolved semi-discrete solution and by its reduction to the plain
scheme when w = 0).
"""
import numpy as np


def leapfrog_step(O, cE, cH, t, dt):
    """One step from (e^n at t, h^{n+1/2}) to (e^{n+1}, h^{n+3/2})."""
    dE, _, _, _ = O.rhs(cE, cH, t=t + 0.5 * dt)
    cE = cE + dt * dE
    _, dH, _, _ = O.rhs(cE, cH, t=t + dt)
    cH = cH + dt * dH
    return cE, cH


def leapfrog_run(O, cE, cH, t0, dt, nsteps):
    t = t0
    for _ in range(nsteps):
        cE, cH = leapfrog_step(O, cE, cH, t, dt)
        t += dt
    return cE, cH, t


def staggered_energy(O, cE, cH_prev, cH_next):
    """1/2 (e, M_eps e) + 1/2 (h_prev, M_mu h_next) in Cartesian coefficients."""
    J = O.J[:, None, None]
    return 0.5 * float(np.sum(J * O.eps[:, None, None] * cE * cE) +
                       np.sum(J * O.mu[:, None, None] * cH_prev * cH_next))


# ---------------------------------------------------------------- with PML
# The damping terms of the PML equations [KS Sec. IV, eqs. p_variable,
# q_variable] taken by the trapezoid rule while the curl terms stay explicit
# (the paper's time scheme, [KS Sec. V]). For a field u (e or h) with material
# m (eps or mu), auxiliary p and undamped derivative k, per Cartesian
# component a of a PML element:
#   (u' - u)/dt = k - eta_a (u' + u)/2 - (p' + p)/(2 m)
#   (p' - p)/dt = -w_a (p' + p)/2 + m xi_a (u' + u)/2
# a 2x2 linear system per component and mode, solved here with a library
# solve. E and p_E live at integer steps, H and p_H at half steps.

def trapezoid_update(O, u, p, k, m, dt):
    """(u', p') of the system above on every element (w = 0 off the PML)."""
    from .dg import pml_tensors
    om = O.omega
    eta, xi = pml_tensors(om)
    h = 0.5 * dt
    mm = m[:, None]
    A = np.empty(om.shape + (2, 2))
    A[..., 0, 0] = 1.0 + h * eta
    A[..., 0, 1] = h / mm
    A[..., 1, 0] = -h * mm * xi
    A[..., 1, 1] = 1.0 + h * om
    b = np.empty(om.shape + (2, u.shape[2]))
    b[..., 0, :] = u + dt * k - h * eta[..., None] * u - (h / mm)[..., None] * p
    b[..., 1, :] = p - h * om[..., None] * p + (h * mm * xi)[..., None] * u
    x = np.linalg.solve(A, b)
    return x[..., 0, :], x[..., 1, :]


def leapfrog_pml_step(O, cE, cH, pE, pH, t, dt):
    """One step (e^n, p_E^n, h^{n+1/2}, p_H^{n+1/2}) -> the same one step later."""
    kE, _, _, _ = O.rhs(cE, cH, t=t + 0.5 * dt, damping=False)
    cE, pE = trapezoid_update(O, cE, pE, kE, O.eps, dt)
    _, kH, _, _ = O.rhs(cE, cH, t=t + dt, damping=False)
    cH, pH = trapezoid_update(O, cH, pH, kH, O.mu, dt)
    return cE, cH, pE, pH


def leapfrog_pml_run(O, cE, cH, pE, pH, t0, dt, nsteps):
    t = t0
    for _ in range(nsteps):
        cE, cH, pE, pH = leapfrog_pml_step(O, cE, cH, pE, pH, t, dt)
        t += dt
    return cE, cH, pE, pH, t
