"""Pins of the oracle's DG operator, PML and RK4 against properties the paper
and the mathematics fix: polynomial consistency, skew-symmetry (energy
conservation of the central flux, Sec. III), the upwind dissipation identity,
PEC compatibility, the covariant mass / curl identities (Sec. II-III), the
PML tensors of the paper's listing and corner formula (Sec. IV, Appendix A),
the RK4 stability polynomial and the point-source limit."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import OracleDG, pml_tensors
from oracle.basis import Dubiner, tet_quadrature

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _jittered_unit(n, seed, amount=0.1):
    verts, tets = W.kuhn_cube_mesh(n, 0.0, 1.0)
    rng = np.random.default_rng(seed)
    verts = W.jitter_interior(verts, 0.0, 1.0, 1.0 / n, amount, rng)
    eps = rng.uniform(1.0, 4.0, size=len(tets))
    mu = rng.uniform(1.0, 2.0, size=len(tets))
    return verts, tets, eps, mu


def _points(O, r=(0.21, 0.33, 0.17)):
    return O.b + np.einsum("kij,j->ki", O.A, np.asarray(r))


# ------------------------------------------------------------ consistency
def _h_poly(x):
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    return np.stack([Y * Y * Z, X * Z * Z, X ** 3 + Y], -1)


def _curl_h_poly(x):
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    return np.stack([1.0 - 2.0 * X * Z, Y * Y - 3.0 * X * X, Z * Z - 2.0 * Y * Z], -1)


def _e_poly(x):
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    return np.stack([Y * Z, X * X, X * Y], -1)


def _curl_e_poly(x):
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    return np.stack([X, 0.0 * Y, 2.0 * X - Z], -1)


@pytest.mark.parametrize("flux", ["central", "upwind"])
def test_polynomial_consistency_interior(flux):
    """Global polynomials of degree <= p: jumps vanish, so the DG operator
    reduces to eps de/dt = curl h, mu dh/dt = -curl e on elements away from
    the boundary (exact up to rounding)."""
    verts, tets, eps, mu = _jittered_unit(3, 1)
    O = OracleDG(verts, tets, 3, eps=eps, mu=mu, flux=flux)
    cE, cH = O.project(_e_poly), O.project(_h_poly)
    dE, dH, _, _ = O.rhs(cE, cH)
    inner = np.all(O.nbr_side >= 0, axis=1)
    assert inner.sum() > 20
    x = _points(O)
    k = np.arange(O.K)
    vE, vH = O.eval_at(dE, k, x), O.eval_at(dH, k, x)
    np.testing.assert_allclose(vE[inner], (_curl_h_poly(x) / eps[:, None])[inner], atol=2e-11)
    np.testing.assert_allclose(vH[inner], (-_curl_e_poly(x) / mu[:, None])[inner], atol=2e-11)


def _e_pec(x):
    # tangential components vanish on every face of the unit cube
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    return np.stack([0.0 * X, X * (1 - X) * Z * (1 - Z), 0.0 * X], -1)


def _curl_e_pec(x):
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    ey_z = X * (1 - X) * (1 - 2 * Z)
    ey_x = (1 - 2 * X) * Z * (1 - Z)
    return np.stack([-ey_z, 0.0 * X, ey_x], -1)


@pytest.mark.parametrize("flux", ["central", "upwind"])
def test_polynomial_consistency_with_pec(flux):
    """With e x n = 0 on the cube boundary, the PEC mirror ghost (Sec. IV) makes
    boundary faces consistent too: exactness on every element (p = 4)."""
    verts, tets, eps, mu = _jittered_unit(2, 2)
    O = OracleDG(verts, tets, 4, eps=eps, mu=mu, flux=flux)
    cE, cH = O.project(_e_pec), O.project(_h_poly)
    dE, dH, _, _ = O.rhs(cE, cH)
    x = _points(O)
    k = np.arange(O.K)
    np.testing.assert_allclose(O.eval_at(dE, k, x), _curl_h_poly(x) / eps[:, None], atol=5e-11)
    np.testing.assert_allclose(O.eval_at(dH, k, x), -_curl_e_pec(x) / mu[:, None], atol=5e-11)


# --------------------------------------------------- energy / skew-symmetry
def test_central_flux_is_skew_adjoint_in_energy_inner_product():
    """Central flux conserves the semi-discrete energy (Sec. III): the operator
    L satisfies <u, M L v> = -<v, M L u> for the mass M = diag(eps J, mu J),
    including heterogeneous eps/mu and PEC faces."""
    verts, tets, eps, mu = _jittered_unit(3, 3)
    O = OracleDG(verts, tets, 3, eps=eps, mu=mu, flux="central")
    rng = np.random.default_rng(0)
    shp = (O.K, 3, O.N)
    m = O.mass_diag()
    for _ in range(3):
        u = [rng.standard_normal(shp), rng.standard_normal(shp)]
        v = [rng.standard_normal(shp), rng.standard_normal(shp)]
        Lu = np.concatenate([x.ravel() for x in O.rhs(*u)[:2]])
        Lv = np.concatenate([x.ravel() for x in O.rhs(*v)[:2]])
        uu = np.concatenate([x.ravel() for x in u])
        vv = np.concatenate([x.ravel() for x in v])
        a = uu @ (m * Lv)
        b = vv @ (m * Lu)
        assert abs(a + b) < 1e-11 * (abs(a) + abs(b))
        assert abs(uu @ (m * Lu)) < 1e-11 * np.linalg.norm(uu) * np.linalg.norm(m * Lu)


def test_upwind_energy_rate_equals_jump_dissipation():
    """dW/dt = -sum_F int |[e]_t|^2/(Z-+Z+) + |[h]_t|^2/(Y-+Y+) dS <= 0 for the
    upwind flux, evaluated by an independent face loop."""
    verts, tets, eps, mu = _jittered_unit(2, 4)
    O = OracleDG(verts, tets, 2, eps=eps, mu=mu, flux="upwind")
    rng = np.random.default_rng(1)
    shp = (O.K, 3, O.N)
    cE, cH = rng.standard_normal(shp), rng.standard_normal(shp)
    dE, dH, _, _ = O.rhs(cE, cH)
    rate = np.sum(O.J[:, None, None] * (O.eps[:, None, None] * cE * dE + O.mu[:, None, None] * cH * dH))
    diss = O.upwind_dissipation(cE, cH)
    assert diss < 0
    assert abs(rate - diss) < 1e-11 * abs(diss)


# ------------------------------------------- covariant identities (Sec. II-III)
def test_covariant_mass_and_geometry_free_curl():
    """Covariant basis A^-T e_j phi_l: mass = J A^-1 A^-T (x) I (Sec. II), and
    (curl phi_jl, phi_km)_T = sign(det A) x the same matrix on every element
    (eq. matrix_free_curl), by physical-space quadrature on two random tets."""
    p = 2
    B = Dubiner(p)
    rq, w = tet_quadrature(p + 2)
    rng = np.random.default_rng(5)
    curls = []
    for trial in range(3):
        X = rng.standard_normal((4, 3))
        A = np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], axis=1)
        Ai = np.linalg.inv(A)
        det = np.linalg.det(A)
        ph = B.eval(rq)  # [Q,N]
        gr = np.einsum("ab,qbm->qam", Ai.T, B.grad(rq))  # physical grads [Q,3,N]
        # covariant vector basis: v_{jl}(x) = A^-T e_j phi_l ; curl = grad phi_l x (A^-T e_j)
        vec = np.einsum("aj,qm->qajm", Ai.T, ph)  # [Q,3(comp),3(j),N]
        # curl(phi_l c_j) = grad phi_l x c_j with the constant vector c_j = A^-T e_j
        cur = np.cross(gr[:, :, None, :], Ai.T[None, :, :, None], axis=1)
        Jw = w * abs(det)
        mass = np.einsum("q,qajl,qakm->jlkm", Jw, vec, vec)
        expect = np.einsum("jk,lm->jlkm", abs(det) * Ai @ Ai.T, np.eye(B.N))
        np.testing.assert_allclose(mass, expect, atol=1e-12 * abs(det) * np.abs(Ai).max() ** 2)
        C = np.einsum("q,qajl,qakm->jlkm", Jw, cur, vec) * np.sign(det)
        curls.append(C)
    np.testing.assert_allclose(curls[1], curls[0], atol=1e-11)
    np.testing.assert_allclose(curls[2], curls[0], atol=1e-11)


# -------------------------------------------------------------------- PML
def test_pml_tensors_match_listing():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "pml_listing_sigma5.txt"))
            if l.strip() and not l.startswith("#")]
    for r in rows:
        w = np.array([float(v) for v in r[1:4]])
        eta, xi = pml_tensors(w)
        np.testing.assert_array_equal(eta, [float(v) for v in r[4:7]])
        np.testing.assert_array_equal(xi, [float(v) for v in r[7:10]])


def test_pml_decomposition_matches_corner_tensor():
    """Sec. IV corner formula eps~_aa = eps s_b s_c / s_a with s_a = 1 + i w_a/omega
    (time dependence e^{-i omega t}) equals eps + i(eta_a eps + xi_a eps/(w_a - i omega))/omega."""
    rng = np.random.default_rng(2)
    for _ in range(20):
        w = rng.uniform(0, 30, 3)
        om = rng.uniform(0.1, 50)
        eta, xi = pml_tensors(w)
        s = 1.0 + 1j * w / om
        for a in range(3):
            b, c = (a + 1) % 3, (a + 2) % 3
            lhs = -1j * om * s[b] * s[c] / s[a]
            rhs = -1j * om + eta[a] + xi[a] / (w[a] - 1j * om)
            assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def test_pml_zero_damping_identical_to_no_pml():
    verts, tets, eps, mu = _jittered_unit(2, 6)
    O0 = OracleDG(verts, tets, 2, eps=eps, mu=mu, flux="upwind")
    O1 = OracleDG(verts, tets, 2, eps=eps, mu=mu, flux="upwind", omega=np.zeros((len(tets), 3)))
    rng = np.random.default_rng(3)
    cE, cH = rng.standard_normal((2, O0.K, 3, O0.N))
    a = O0.rhs(cE, cH)
    b = O1.rhs(cE, cH, np.zeros_like(cE), np.zeros_like(cH))
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_pml_auxiliary_relaxes_with_own_pole():
    """With xi = 0 (equal damping on all axes, the corner region of Sec. IV) the
    auxiliary decouples from e: d_t p_a = -w_a p_a (eq. p_variable), so one RK4
    step multiplies it by R(-w_a dt)."""
    verts, tets, eps, mu = _jittered_unit(2, 7)
    rng = np.random.default_rng(4)
    z = np.zeros((len(tets), 3, 10))
    pE, pH = rng.standard_normal((2, len(tets), 3, 10))
    dt = 0.01
    om2 = np.repeat(rng.uniform(0, 20, (len(tets), 1)), 3, axis=1)
    O2 = OracleDG(verts, tets, 2, eps=eps, mu=mu, flux="central", omega=om2)
    (_, _, pE2, _), _ = O2.run(z, z, pE, pH, dt=dt, nsteps=1)
    x2 = -om2 * dt
    R2 = 1 + x2 + x2 ** 2 / 2 + x2 ** 3 / 6 + x2 ** 4 / 24
    np.testing.assert_allclose(pE2, R2[:, :, None] * pE, rtol=1e-13, atol=1e-13)


# -------------------------------------------------------------------- RK4
def test_rk4_step_is_stability_polynomial():
    """One RK4 step of a linear autonomous system equals R(dt L) u with
    R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24."""
    verts, tets = W.kuhn_cube_mesh(1, 0.0, 1.0)
    O = OracleDG(verts, tets, 1, flux="upwind", eps=np.linspace(1, 2, 6))
    L = O.assemble()
    rng = np.random.default_rng(8)
    u = rng.standard_normal(L.shape[0])
    dt = 0.05
    Z = dt * L
    R = np.eye(len(u)) + Z + Z @ Z / 2 + Z @ Z @ Z / 6 + Z @ Z @ Z @ Z / 24
    n = O.K * 3 * O.N
    (cE, cH, _, _), _ = O.run(u[:n].reshape(O.K, 3, O.N).copy(), u[n:].reshape(O.K, 3, O.N).copy(), dt=dt)
    np.testing.assert_allclose(np.concatenate([cE.ravel(), cH.ravel()]), R @ u, rtol=1e-12, atol=1e-12)


# ----------------------------------------------------------------- source
def test_point_source_is_limit_of_narrow_gaussian():
    """-(j, v) for j = d delta(r-r0) g(t) equals the limit w -> 0 of the
    projected smooth current d g(t) G_w(r - r0) (error O(w^2))."""
    verts, tets = W.kuhn_cube_mesh(2, 0.0, 1.0)
    O = OracleDG(verts, tets, 2, flux="central")
    k0 = 17
    r0 = O.b[k0] + O.A[k0] @ np.array([0.24, 0.26, 0.23])
    d = np.array([0.3, -0.5, 0.8])
    gval = 0.7
    Od = OracleDG(verts, tets, 2, flux="central", dipoles=[(r0, d, lambda t: gval)])
    z = np.zeros((O.K, 3, O.N))
    dE, _, _, _ = Od.rhs(z, z, t=0.0)
    assert np.abs(np.delete(dE, k0, axis=0)).max() == 0.0
    # smoothed current d g G_w(r - r0); (j_w, phi_m)_T = E[phi_m(r0 + w Z)] over
    # Z ~ N(0, I), computed with a tensor Gauss-Hermite rule (the Gaussian mass
    # outside the element is negligible at these widths)
    from scipy.special import roots_hermitenorm
    z1, w1 = roots_hermitenorm(8)
    w1 = w1 / np.sqrt(2 * np.pi)
    Z3 = np.stack(np.meshgrid(z1, z1, z1, indexing="ij"), -1).reshape(-1, 3)
    W3 = np.einsum("i,j,k->ijk", w1, w1, w1).ravel()
    exps = []
    for w in (0.02, 0.01):
        x = r0 + w * Z3
        ph = O.basis.eval(np.einsum("ij,qj->qi", O.Ainv[k0], x - O.b[k0]))  # [Q,N]
        integ = np.einsum("q,qm->m", W3, ph)
        exps.append(-gval * np.outer(d, integ) / (O.eps[k0] * O.J[k0]))
    # for p = 2 the smoothing error is exactly quadratic in w (heat kernel of a
    # quadratic), so Richardson extrapolation to w = 0 is exact
    limit = (4.0 * exps[1] - exps[0]) / 3.0
    assert np.abs(exps[1] - dE[k0]).max() > 1e-4  # the smoothing is visible
    np.testing.assert_allclose(dE[k0], limit, rtol=0, atol=1e-10 * np.abs(dE[k0]).max())
