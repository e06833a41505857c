"""Pins of the oracle's discrete adjoint (test infrastructure for the GPU
adjoint): its gradient of the probe energy with respect to every element's
permittivity against central finite differences of the oracle's own RK4
objective, and its J against the plain trajectory."""
import numpy as np

import workloads as W
from oracle import OracleDG
from oracle.adjoint import adjoint_gradient, probe_objective


def _problem(eps, omega=None, flux="central"):
    verts, tets = W.kuhn_cube_mesh(2, 0.0, 1.0)
    rng = np.random.default_rng(41)
    verts = W.jitter_interior(verts, 0.0, 1.0, 0.5, 0.1, rng)
    dip = [(np.array([0.4, 0.45, 0.55]), np.array([0.3, 0.2, 1.0]),
            lambda t: W.dipole_waveform(t, 2.0, 1.0))]
    mu = np.linspace(1.0, 2.0, len(tets))  # impedances differ across faces
    return OracleDG(verts, tets, 1, eps=eps, mu=mu, flux=flux, dipoles=dip, omega=omega)


def test_oracle_adjoint_matches_finite_differences():
    rng = np.random.default_rng(42)
    eps = rng.uniform(1.0, 4.0, 48)
    O = _problem(eps)
    cE0 = 0.3 * rng.standard_normal((48, 3, O.N))
    cH0 = 0.3 * rng.standard_normal((48, 3, O.N))
    dt, nsteps, probes = 0.01, 8, np.array([3, 17, 40])
    J, g = adjoint_gradient(O, cE0, cH0, dt, nsteps, probes)
    assert abs(J - probe_objective(O, cE0, cH0, dt, nsteps, probes)) < 1e-12 * abs(J)
    for T in (0, 3, 17, 29, 40, 47):
        h = 1e-5 * eps[T]
        ep, em = eps.copy(), eps.copy()
        ep[T] += h
        em[T] -= h
        # the initial state is held in Cartesian coefficients: the fields
        # themselves are fixed while eps moves
        Jp = probe_objective(_problem(ep), cE0, cH0, dt, nsteps, probes)
        Jm = probe_objective(_problem(em), cE0, cH0, dt, nsteps, probes)
        fd = (Jp - Jm) / (2 * h)
        assert abs(g[T] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()), (T, g[T], fd)


def test_oracle_adjoint_with_pml_matches_finite_differences():
    """PML elements (per-axis poles, one axis undamped on some): eps enters
    the curl terms, eta/xi couplings and the auxiliary equation; the
    auxiliaries start at zero."""
    rng = np.random.default_rng(43)
    eps = rng.uniform(1.0, 4.0, 48)
    omega = np.zeros((48, 3))
    sel = rng.random(48) < 0.5
    omega[sel] = rng.uniform(1.0, 8.0, (sel.sum(), 3))
    omega[sel & (rng.random(48) < 0.4), 2] = 0.0
    O = _problem(eps, omega)
    cE0 = 0.3 * rng.standard_normal((48, 3, O.N))
    cH0 = 0.3 * rng.standard_normal((48, 3, O.N))
    dt, nsteps, probes = 0.01, 8, np.array([3, 17, 40])
    J, g = adjoint_gradient(O, cE0, cH0, dt, nsteps, probes)
    assert abs(J - probe_objective(O, cE0, cH0, dt, nsteps, probes)) < 1e-12 * abs(J)
    checked = 0
    for T in (0, 3, 17, 29, 40, 47) + tuple(np.flatnonzero(sel)[:4]):
        h = 1e-5 * eps[T]
        ep, em = eps.copy(), eps.copy()
        ep[T] += h
        em[T] -= h
        Jp = probe_objective(_problem(ep, omega), cE0, cH0, dt, nsteps, probes)
        Jm = probe_objective(_problem(em, omega), cE0, cH0, dt, nsteps, probes)
        fd = (Jp - Jm) / (2 * h)
        assert abs(g[T] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()), (T, g[T], fd)
        checked += int(sel[T])
    assert checked >= 4


def test_operator_difference_derivative_matches_analytic():
    """The eps-derivative of the stage derivatives taken by central
    differences of the operator (the route used for the upwind flux) against
    the closed form of the central flux with PML."""
    rng = np.random.default_rng(44)
    eps = rng.uniform(1.0, 4.0, 48)
    omega = np.zeros((48, 3))
    omega[rng.random(48) < 0.5] = 3.0
    O = _problem(eps, omega)
    cE0 = 0.3 * rng.standard_normal((48, 3, O.N))
    cH0 = 0.3 * rng.standard_normal((48, 3, O.N))
    Ja, ga = adjoint_gradient(O, cE0, cH0, 0.01, 6, np.array([3, 40]), deps="analytic")
    Jf, gf = adjoint_gradient(O, cE0, cH0, 0.01, 6, np.array([3, 40]), deps="fd")
    assert Ja == Jf
    assert np.abs(ga - gf).max() < 1e-7 * np.abs(ga).max()


def test_oracle_adjoint_upwind_matches_finite_differences():
    """Upwind flux (eps in the impedances of every face of T and of its
    neighbours' equations) with PML elements: the adjoint gradient against
    central finite differences of the objective."""
    rng = np.random.default_rng(45)
    eps = rng.uniform(1.0, 4.0, 48)
    omega = np.zeros((48, 3))
    sel = rng.random(48) < 0.4
    omega[sel] = rng.uniform(1.0, 6.0, (sel.sum(), 3))
    O = _problem(eps, omega, "upwind")
    cE0 = 0.3 * rng.standard_normal((48, 3, O.N))
    cH0 = 0.3 * rng.standard_normal((48, 3, O.N))
    dt, nsteps, probes = 0.01, 8, np.array([3, 17, 40])
    J, g = adjoint_gradient(O, cE0, cH0, dt, nsteps, probes)
    assert abs(J - probe_objective(O, cE0, cH0, dt, nsteps, probes)) < 1e-12 * abs(J)
    for T in (0, 3, 17, 22, 40, 47) + tuple(np.flatnonzero(sel)[:3]):
        h = 1e-5 * eps[T]
        ep, em = eps.copy(), eps.copy()
        ep[T] += h
        em[T] -= h
        Jp = probe_objective(_problem(ep, omega, "upwind"), cE0, cH0, dt, nsteps, probes)
        Jm = probe_objective(_problem(em, omega, "upwind"), cE0, cH0, dt, nsteps, probes)
        fd = (Jp - Jm) / (2 * h)
        assert abs(g[T] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()), (T, g[T], fd)
