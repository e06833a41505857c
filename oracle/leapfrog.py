"""Test infrastructure: the staggered leap-frog time scheme the paper uses for
its experiments [KS Sec. V] with the oracle's operator, written plainly.

State (e^n, h^{n+1/2}). With the central flux the E derivative depends only
on h (and the current j) and the H derivative only on e, so one step is
    e^{n+1}   = e^n       + dt dE(h^{n+1/2}, t^{n+1/2})
    h^{n+3/2} = h^{n+1/2} + dt dH(e^{n+1})
The quantity W^n = 1/2 (e^n, M_eps e^n) + 1/2 (h^{n-1/2}, M_mu h^{n+1/2}) is
conserved exactly without sources (pinned in tests/test_oracle_leapfrog.py).
Equal orders for e and h, no PML (the paper's trapezoidal treatment of the
damping terms and its mixed orders are not part of this scheme).
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
