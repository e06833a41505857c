"""Pins of the oracle's leap-frog scheme (test infrastructure for the
library's leap-frog integrator): the staggered energy is conserved to
round-off with the central flux, and the time error is second order."""
import numpy as np

import workloads as W
from oracle import OracleDG
from oracle.leapfrog import leapfrog_run, leapfrog_step, staggered_energy


def test_staggered_energy_is_conserved():
    verts, tets = W.kuhn_cube_mesh(2, 0.0, 1.0)
    rng = np.random.default_rng(3)
    verts = W.jitter_interior(verts, 0.0, 1.0, 0.5, 0.1, rng)
    eps, mu = rng.uniform(1, 4, 48), rng.uniform(1, 2, 48)
    O = OracleDG(verts, tets, 2, eps=eps, mu=mu, flux="central")
    cE = rng.standard_normal((48, 3, O.N))
    cH = rng.standard_normal((48, 3, O.N))
    dt = 2e-3
    # h^{-1/2} from h^{1/2} by one backward half of the step
    _, dH, _, _ = O.rhs(cE, cH)
    h_prev = cH - dt * dH
    W0 = staggered_energy(O, cE, h_prev, cH)
    for _ in range(150):
        h_prev = cH
        cE, cH = leapfrog_step(O, cE, cH, 0.0, dt)
    W1 = staggered_energy(O, cE, h_prev, cH)
    assert abs(W1 - W0) < 1e-12 * W0


def test_leapfrog_is_second_order_in_time():
    w = W.cavity(2, 2)
    O = OracleDG(w.verts, w.tets, 2, flux="central")
    rng = np.random.default_rng(5)
    cE0 = rng.standard_normal((w.nt, 3, O.N))
    cH0 = rng.standard_normal((w.nt, 3, O.N))
    T = 0.08
    # reference: the same semi-discrete system by RK4 with a tiny step; the
    # leap-frog h starts half a step late, so compare e only
    ref = O.run(cE0, cH0, dt=T / 800, nsteps=800)[0][0]
    errs = []
    for n in (20, 40, 80):
        dt = T / n
        # h^{1/2} from h^0 by RK4 over half a step (second-order accurate start)
        hh = O.run(cE0, cH0, dt=0.5 * dt / 8, nsteps=8)[0][1]
        e, _, _ = leapfrog_run(O, cE0, hh, 0.0, dt, n)
        errs.append(np.sqrt(np.sum(O.J[:, None, None] * (e - ref) ** 2)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, (errs, r1, r2)
