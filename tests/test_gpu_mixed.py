"""GPU parity of the mixed orders (e at order p+1, h at order p, the paper's
pairing [KS eqs. triale, trialh]) against the oracle's mixed-order operator
(OracleDG(..., p + 1, ph=p)), which builds both spaces from their own bases.

* Operator: central and upwind, with PML elements and a dipole, FP64 and
  FP32, on meshes of several tiles.
* RK4 trajectory (upwind, PML, dipole) and the paper's own scheme: leap-frog
  with trapezoid PML damping and mixed orders; staggered energy conservation
  without PML.
* State round trip and L2 projection of h into its own (lower) space.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_helpers import dipole_args, oracle_dipoles, rel_energy_err, say, unit_jittered

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_08733_amd import load_library
    load_library()


def _pair(verts, tets, p, flux, precision, eps, mu, omega=None, dipoles=(), dt=1e-3, integrator="rk4"):
    from oracle import OracleDG
    from paper_2002_08733_amd import Solver
    s = Solver(p, precision, flux, dt=dt, integrator=integrator, mixed=True)
    s.set_mesh(verts, tets)
    s.set_material(eps, mu)
    if omega is not None:
        s.set_pml(omega)
    if dipoles:
        s.set_dipoles(*dipole_args(dipoles))
    s.bind_torch_workspace()
    O = OracleDG(verts, tets, p + 1, eps=eps, mu=mu, flux=flux, omega=omega, dipoles=oracle_dipoles(dipoles), ph=p)
    assert (s.nmodes, s.nmodes_h) == (O.N, O.NH)
    return s, O


def _pml_omega(verts, tets, rng):
    c = W.tet_centroids(verts, tets)
    omega = np.zeros((len(tets), 3))
    sel = c[:, 2] > 0.6
    omega[sel] = rng.uniform(1.0, 5.0, (sel.sum(), 3))
    omega[sel & (c[:, 0] < 0.3), 1] = 0.0
    return omega, sel


def _dip():
    return [(np.array([0.45, 0.5, 0.52]), np.array([0.1, 0.3, 0.95]), (2.0, 1.0))]


@pytest.mark.parametrize("p,flux,precision,tol", [
    (2, "central", "fp64", 1e-12), (2, "upwind", "fp64", 1e-12), (3, "upwind", "fp64", 1e-12),
    (2, "upwind", "fp32", 2e-5), (3, "central", "fp32", 2e-5)])
def test_mixed_operator_parity(p, flux, precision, tol):
    verts, tets, eps, mu = unit_jittered(4, 51 + p)
    rng = np.random.default_rng(52)
    omega, pml = _pml_omega(verts, tets, rng)
    s, O = _pair(verts, tets, p, flux, precision, eps, mu, omega, _dip())
    K = len(tets)
    uE, uP = rng.standard_normal((K, 3, O.N)), rng.standard_normal((K, 3, O.N))
    uH, uQ = rng.standard_normal((K, 3, O.NH)), rng.standard_normal((K, 3, O.NH))
    uP[~pml] = 0.0
    uQ[~pml] = 0.0
    t = 0.8
    say(f"[mixed rhs] e order {p + 1}, h order {p}, {flux} {precision}: K={K} ({pml.sum()} PML), "
        f"{s.query()['n_tiles']} tiles")
    dE, dH, dP, dQ = s.rhs(uE, uH, uP, uQ, t=t, aux=True)
    s.close()
    cv = O.to_cartesian
    oE, oH, oP, oQ = O.rhs(cv(uE), cv(uH), cv(uP), cv(uQ), t=t)
    oP[~pml] = 0.0
    oQ[~pml] = 0.0
    err = rel_energy_err(O, cv(dE), cv(dH), oE, oH, cv(dP), cv(dQ), oP, oQ)
    say(f"  rel err {err:.3e}")
    assert dH.shape == (K, 3, O.NH) and err < tol


def test_mixed_rk4_trajectory_with_pml():
    verts, tets, eps, mu = unit_jittered(4, 55)
    rng = np.random.default_rng(56)
    omega, pml = _pml_omega(verts, tets, rng)
    s, O = _pair(verts, tets, 2, "upwind", "fp64", eps, mu, omega, _dip(), dt=2e-3)
    K = len(tets)
    E0, H0 = rng.standard_normal((K, 3, O.N)), rng.standard_normal((K, 3, O.NH))
    s.set_state(E0, H0, t=0.5)
    s.step(8)
    E, H, P, Q, t = s.get_state(aux=True)
    s.close()
    cv = O.to_cartesian
    (cE, cH, cP, cQ), to = O.run(cv(E0), cv(H0), t0=0.5, dt=2e-3, nsteps=8)
    err = rel_energy_err(O, cv(E), cv(H), cE, cH, cv(P), cv(Q), cP, cQ)
    say(f"[mixed RK4] e3/h2 upwind + PML + dipole, 8 steps: rel err {err:.3e}")
    assert abs(t - to) < 1e-12 and err < 1e-12


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_mixed_leapfrog_trapezoid_pml(precision, tol):
    """The paper's scheme: mixed orders, leap-frog, PML damping by the
    trapezoid rule, a dipole at the half steps."""
    from oracle.leapfrog import leapfrog_pml_run
    verts, tets, eps, mu = unit_jittered(5, 57)
    rng = np.random.default_rng(58)
    omega, pml = _pml_omega(verts, tets, rng)
    dt = W.cfl_dt(verts, tets, eps, mu, 3, 0.2)
    s, O = _pair(verts, tets, 2, "central", precision, eps, mu, omega, _dip(), dt=dt, integrator="leapfrog")
    K = len(tets)
    E0, P0 = rng.standard_normal((K, 3, O.N)), rng.standard_normal((K, 3, O.N))
    H0, Q0 = rng.standard_normal((K, 3, O.NH)), rng.standard_normal((K, 3, O.NH))
    P0[~pml] = 0.0
    Q0[~pml] = 0.0
    s.set_state(E0, H0, P0, Q0, t=0.6)
    s.step(20)
    E, H, P, Q, _ = s.get_state(aux=True)
    s.close()
    cv = O.to_cartesian
    cE, cH, cP, cQ, _ = leapfrog_pml_run(O, cv(E0), cv(H0), cv(P0), cv(Q0), 0.6, dt, 20)
    err = rel_energy_err(O, cv(E), cv(H), cE, cH, cv(P), cv(Q), cP, cQ)
    say(f"[mixed leap-frog] e3/h2 central + trapezoid PML + dipole {precision}, K={K}, 20 steps: rel err {err:.3e}")
    assert err < tol


def test_mixed_leapfrog_staggered_energy():
    from oracle.leapfrog import staggered_energy
    verts, tets, eps, mu = unit_jittered(5, 59)
    dt = W.cfl_dt(verts, tets, eps, mu, 4, 0.2)
    s, O = _pair(verts, tets, 3, "central", "fp64", eps, mu, dt=dt, integrator="leapfrog")
    rng = np.random.default_rng(60)
    K = len(tets)
    s.set_state(rng.standard_normal((K, 3, O.N)), rng.standard_normal((K, 3, O.NH)))
    cv = O.to_cartesian

    def w_next():
        _, Hp, _ = s.get_state()
        s.step(1)
        E, H, _ = s.get_state()
        return staggered_energy(O, cv(E), cv(Hp), cv(H))

    W1 = w_next()
    s.step(150)
    W2 = w_next()
    s.close()
    say(f"[mixed leap-frog energy] e4/h3: W {W1:.15e} -> {W2:.15e} ({(W2 - W1) / W1:.1e})")
    assert abs(W2 - W1) < 1e-12 * W1


def test_mixed_state_roundtrip_and_projection():
    from paper_2002_08733_amd import Solver
    from oracle import OracleDG
    verts, tets, eps, mu = unit_jittered(3, 61)
    s = Solver(2, "fp64", "upwind", dt=1e-3, mixed=True)
    s.set_mesh(verts, tets)
    s.set_material(eps, mu)
    s.bind_torch_workspace()
    O = OracleDG(verts, tets, 3, eps=eps, mu=mu, ph=2)
    rng = np.random.default_rng(62)
    K = len(tets)
    E0, H0 = rng.standard_normal((K, 3, O.N)), rng.standard_normal((K, 3, O.NH))
    s.set_state(E0, H0)
    E, H, _ = s.get_state()
    assert np.array_equal(E, E0) and np.array_equal(H, H0)
    # cubic fields: both quadratures are exact, and h (order 2) keeps only
    # its projection onto P_2
    def fe(y):
        return np.stack([y[..., 0] * y[..., 1], y[..., 1] * y[..., 2] ** 2, y[..., 0] ** 3 - y[..., 2]], axis=-1)

    def fh(y):
        return np.stack([y[..., 2] * y[..., 0] ** 2, y[..., 0] * y[..., 1] * y[..., 2], y[..., 1] ** 3], axis=-1)

    x = s.projection_points(6)
    s.project(6, fe(x), fh(x))
    E, H, _ = s.get_state()
    W_lib = s.energy()
    s.close()
    oE = O.project(fe)
    oH = O.project(fh, field="h")
    dE = np.abs(O.to_cartesian(E) - oE).max() / np.abs(oE).max()
    dH = np.abs(O.to_cartesian(H) - oH).max() / np.abs(oH).max()
    say(f"[mixed projection] e3/h2: max rel diff E {dE:.2e}, H {dH:.2e}; energy {W_lib:.9e} vs {O.energy(oE, oH):.9e}")
    assert dE < 1e-10 and dH < 1e-10
    assert abs(W_lib - O.energy(oE, oH)) < 1e-10 * W_lib
