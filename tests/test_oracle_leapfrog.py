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


def _pml_problem(seed):
    verts, tets = W.kuhn_cube_mesh(2, 0.0, 1.0)
    rng = np.random.default_rng(seed)
    verts = W.jitter_interior(verts, 0.0, 1.0, 0.5, 0.1, rng)
    K = len(tets)
    eps, mu = rng.uniform(1, 3, K), rng.uniform(1, 2, K)
    omega = np.zeros((K, 3))
    pml = rng.random(K) < 0.5
    omega[pml] = rng.uniform(1.0, 6.0, (pml.sum(), 3))
    omega[pml & (rng.random(K) < 0.3), 1] = 0.0  # edge-type elements
    return verts, tets, eps, mu, omega, pml, rng


def test_trapezoid_leapfrog_reduces_to_plain_without_damping():
    from oracle.leapfrog import leapfrog_pml_step
    verts, tets, eps, mu, _, _, rng = _pml_problem(11)
    K = len(tets)
    O = OracleDG(verts, tets, 2, eps=eps, mu=mu, flux="central", omega=np.zeros((K, 3)))
    shp = (K, 3, O.N)
    cE, cH = rng.standard_normal(shp), rng.standard_normal(shp)
    z = np.zeros(shp)
    e1, h1, p1, q1 = leapfrog_pml_step(O, cE, cH, z, z, 0.0, 3e-3)
    O0 = OracleDG(verts, tets, 2, eps=eps, mu=mu, flux="central")
    e0, h0 = leapfrog_step(O0, cE, cH, 0.0, 3e-3)
    assert np.abs(e1 - e0).max() < 1e-14 * np.abs(e0).max()
    assert np.abs(h1 - h0).max() < 1e-14 * np.abs(h0).max()
    assert not p1.any() and not q1.any()


def test_trapezoid_leapfrog_with_pml_is_second_order():
    """The scheme converges at second order to the semi-discrete PML system
    (resolved by RK4 with a tiny step), whose damping changes the solution by
    far more than the leap-frog errors: a wrong damping term fails here."""
    from oracle.leapfrog import leapfrog_pml_run
    verts, tets, eps, mu, omega, pml, rng = _pml_problem(12)
    K = len(tets)
    O = OracleDG(verts, tets, 2, eps=eps, mu=mu, flux="central", omega=omega)
    shp = (K, 3, O.N)
    cE0, cH0 = rng.standard_normal(shp), rng.standard_normal(shp)
    pE0, pH0 = rng.standard_normal(shp), rng.standard_normal(shp)
    pE0[~pml] = 0.0
    pH0[~pml] = 0.0
    T = 0.12
    (rE, _, rP, _), _ = O.run(cE0, cH0, pE0, pH0, dt=T / 960, nsteps=960)
    O0 = OracleDG(verts, tets, 2, eps=eps, mu=mu, flux="central")
    (nE, _, _, _), _ = O0.run(cE0, cH0, dt=T / 960, nsteps=960)

    def norm(e, p):
        return np.sqrt(np.sum(O.J[:, None, None] * (e * e + p * p)))

    errs = []
    for n in (15, 30, 60):
        dt = T / n
        (_, hh, _, qh), _ = O.run(cE0, cH0, pE0, pH0, dt=0.5 * dt / 8, nsteps=8)
        e, _, p, _, _ = leapfrog_pml_run(O, cE0, hh, pE0, qh, 0.0, dt, n)
        errs.append(norm(e - rE, p - rP))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, (errs, r1, r2)
    assert errs[-1] < 0.02 * norm(rE - nE, rP)
