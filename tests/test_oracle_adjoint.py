"""Pins of the oracle's discrete adjoint (test infrastructure for the GPU
adjoint): its gradient of the probe energy with respect to every element's
permittivity against central finite differences of the oracle's own RK4
objective, and its J against the plain trajectory."""
import numpy as np

import workloads as W
from oracle import OracleDG
from oracle.adjoint import adjoint_gradient, probe_objective


def _problem(eps, omega=None, flux="central"):
    """2^3 Kuhn cubes (48 tets) of the unit cube, jittered, p = 1, mu varying
    across elements, a dipole."""
    verts, tets = W.kuhn_cube_mesh(2, 0.0, 1.0)
    rng = np.random.default_rng(41)
    verts = W.jitter_interior(verts, 0.0, 1.0, 0.5, 0.1, rng)
    dip = [(np.array([0.4, 0.45, 0.55]), np.array([0.3, 0.2, 1.0]),
            lambda t: W.dipole_waveform(t, 2.0, 1.0))]
    mu = np.linspace(1.0, 2.0, len(tets))  # impedances differ across faces
    return OracleDG(verts, tets, 1, eps=eps, mu=mu, flux=flux, dipoles=dip, omega=omega)


def _one_cube(eps, omega=None, flux="central"):
    """One cube of 6 tets with every vertex moved (all faces stay conforming;
    12 PEC faces, 6 interior), p = 1, mu varying, a dipole."""
    verts, tets = W.kuhn_cube_mesh(1, 0.0, 1.0)
    verts = verts + 0.06 * np.random.default_rng(48).standard_normal(verts.shape)
    dip = [(np.array([0.45, 0.5, 0.55]), np.array([0.3, 0.2, 1.0]), lambda t: W.dipole_waveform(t, 2.0, 1.0))]
    mu = np.linspace(1.0, 2.0, len(tets))
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


def test_complex_step_derivative_matches_analytic():
    """The eps-derivative of the stage derivatives by complex steps of the
    operator (the route used for the upwind flux) against the closed form of
    the central flux with PML: the same gradient to rounding."""
    rng = np.random.default_rng(44)
    eps = rng.uniform(1.0, 4.0, 48)
    omega = np.zeros((48, 3))
    omega[rng.random(48) < 0.5] = 3.0
    O = _problem(eps, omega)
    cE0 = 0.3 * rng.standard_normal((48, 3, O.N))
    cH0 = 0.3 * rng.standard_normal((48, 3, O.N))
    Ja, ga = adjoint_gradient(O, cE0, cH0, 0.01, 6, np.array([3, 40]), deps="analytic")
    Jc, gc = adjoint_gradient(O, cE0, cH0, 0.01, 6, np.array([3, 40]), deps="complex")
    assert Ja == Jc
    assert np.abs(ga - gc).max() < 1e-13 * np.abs(ga).max()


def test_complex_step_of_the_upwind_operator_matches_differences():
    """Complex step of the upwind operator by eps_T on T and its neighbours
    against a fourth-order central difference of the real operator (an
    independent route with truncation ~1e-12 at this step)."""
    from oracle.adjoint import _with_complex_eps
    rng = np.random.default_rng(46)
    eps = rng.uniform(1.0, 4.0, 48)
    O = _problem(eps, flux="upwind")
    cE = rng.standard_normal((48, 3, O.N))
    cH = rng.standard_normal((48, 3, O.N))
    for T in (0, 21, 47):
        el = np.array([T] + [sd // 4 for sd in O.nbr_side[T] if sd >= 0])
        d = 1e-20 * eps[T]
        dE, dH, _, _ = _with_complex_eps(O, T, d).rhs(cE, cH, elems=el, t=0.3)
        cs = np.concatenate([dE.imag.ravel(), dH.imag.ravel()]) / d

        def real_at(x):
            e = eps.copy()
            e[T] = x
            Oe = _problem(e, flux="upwind")
            a, b, _, _ = Oe.rhs(cE, cH, elems=el, t=0.3)
            return np.concatenate([a.ravel(), b.ravel()])
        h = 2e-3 * eps[T]
        fd = (-real_at(eps[T] + 2 * h) + 8 * real_at(eps[T] + h) - 8 * real_at(eps[T] - h)
              + real_at(eps[T] - 2 * h)) / (12 * h)
        assert np.abs(cs - fd).max() < 1e-9 * np.abs(cs).max(), T
        assert np.abs(cs).max() > 0


def test_oracle_adjoint_with_sip_matches_finite_differences():
    """Central flux with the SIP surface unknown h_s [KS Sec. III] and PML
    elements: the state carries h_s from zero, eps enters only the E rows
    (mass inverse of every E term, h_s coupling included) and the PML terms.
    The adjoint gradient against central differences of the SIP oracle's own
    RK4 objective, and the analytic route against the complex-step route."""
    from oracle.sip import SipDG
    rng = np.random.default_rng(47)
    K = 6
    eps = rng.uniform(1.0, 4.0, K)
    omega = np.zeros((K, 3))
    sel = np.array([True, False, True, False, False, True])
    omega[sel] = rng.uniform(1.0, 6.0, (sel.sum(), 3))
    _problem = _one_cube
    O = _problem(eps, omega)
    sip = SipDG(O, 1.0)
    cE0 = 0.3 * rng.standard_normal((K, 3, O.N))
    cH0 = 0.3 * rng.standard_normal((K, 3, O.N))
    dt, nsteps, probes = 0.005, 6, np.array([1, 4])
    J, g = adjoint_gradient(O, cE0, cH0, dt, nsteps, probes, sip=sip)
    assert abs(J - probe_objective(O, cE0, cH0, dt, nsteps, probes, sip=sip)) < 1e-12 * abs(J)
    Jc, gc = adjoint_gradient(O, cE0, cH0, dt, nsteps, probes, sip=sip, deps="complex")
    assert np.abs(g - gc).max() < 1e-13 * np.abs(g).max()
    # h_s matters: the gradient without it differs
    _, g0 = adjoint_gradient(O, cE0, cH0, dt, nsteps, probes)
    assert np.abs(g - g0).max() > 1e-3 * np.abs(g).max()
    for T in range(K):
        h = 1e-5 * eps[T]
        ep, em = eps.copy(), eps.copy()
        ep[T] += h
        em[T] -= h
        Op, Om = _problem(ep, omega), _problem(em, omega)
        Jp = probe_objective(Op, cE0, cH0, dt, nsteps, probes, sip=SipDG(Op, 1.0))
        Jm = probe_objective(Om, cE0, cH0, dt, nsteps, probes, sip=SipDG(Om, 1.0))
        fd = (Jp - Jm) / (2 * h)
        # the differences carry ~1e-9 max|g| of rounding (elements far from
        # the probes have gradients 1e-4 of the largest)
        assert abs(g[T] - fd) <= max(1e-6 * abs(fd), 1e-8 * np.abs(g).max()), (T, g[T], fd)


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
