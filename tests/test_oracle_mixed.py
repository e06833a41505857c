"""Pins of the oracle's mixed orders: e at order p+1 and h at order p, the
paper's pairing [KS eqs. triale, trialh].

* Nested spaces: the orthonormal Dubiner modes of P_p are, in the mode order
  used (total degree first), the first dim P_p modes of P_{p+1}, and the mass
  is diagonal in the modes. So with h in P_p the mixed system's E derivative
  equals that of the equal-order (p+1) system with h padded by zeros, and its
  H derivative is the first dim P_p modes of the equal-order H derivative
  (the mixed H equation is tested with a subset of the test functions).
  Checked with central and upwind fluxes, PML elements and a dipole; the
  equal-order oracle is pinned on its own (test_oracle_operator.py,
  test_oracle_physics.py).
* Central flux: the mixed operator is skew in the energy inner product,
  u . M_eps du + f . M_mu df = 0 for any state (the weak E curl and the
  strong H curl with the consistent face term are adjoint [KS Sec. III]).
* TE101 cavity: the mixed pairing converges, and its error lies below that
  of equal orders at the lower order.
"""
import numpy as np
import pytest

import workloads as W
from oracle import OracleDG
from oracle.basis import Dubiner


def _mesh(seed, n=2):
    verts, tets = W.kuhn_cube_mesh(n, 0.0, 1.0)
    rng = np.random.default_rng(seed)
    verts = W.jitter_interior(verts, 0.0, 1.0, 1.0 / n, 0.1, rng)
    K = len(tets)
    return verts, tets, rng.uniform(1, 4, K), rng.uniform(1, 2, K), rng


def test_dubiner_modes_are_nested():
    rng = np.random.default_rng(1)
    r = rng.dirichlet(np.ones(4), 50)[:, 1:]
    for p in (1, 2, 3):
        lo, hi = Dubiner(p).eval(r), Dubiner(p + 1).eval(r)
        assert np.array_equal(lo, hi[:, :lo.shape[1]])


@pytest.mark.parametrize("flux", ["central", "upwind"])
@pytest.mark.parametrize("ph", [1, 2])
def test_mixed_equals_equal_order_with_h_in_the_lower_space(flux, ph):
    verts, tets, eps, mu, rng = _mesh(3 + ph)
    K = len(tets)
    omega = np.zeros((K, 3))
    sel = rng.random(K) < 0.4
    omega[sel] = rng.uniform(0.5, 4.0, (sel.sum(), 3))
    dip = [(np.array([0.4, 0.55, 0.45]), np.array([0.2, 0.3, 0.9]), lambda t: np.sin(3.0 * t) + 0.5)]
    Om = OracleDG(verts, tets, ph + 1, eps=eps, mu=mu, flux=flux, omega=omega, dipoles=dip, ph=ph)
    Oe = OracleDG(verts, tets, ph + 1, eps=eps, mu=mu, flux=flux, omega=omega, dipoles=dip)
    N, NH = Om.N, Om.NH
    assert (N, NH) == (Oe.N, Dubiner(ph).N)
    cE, pE = rng.standard_normal((K, 3, N)), rng.standard_normal((K, 3, N))
    cH, pH = rng.standard_normal((K, 3, NH)), rng.standard_normal((K, 3, NH))

    def pad(a):
        out = np.zeros((K, 3, N))
        out[:, :, :NH] = a
        return out

    m = Om.rhs(cE, cH, pE, pH, t=0.3)
    e = Oe.rhs(cE, pad(cH), pE, pad(pH), t=0.3)
    for a, b in ((m[0], e[0]), (m[2], e[2]), (m[1], e[1][:, :, :NH]), (m[3], e[3][:, :, :NH])):
        assert a.shape == b.shape
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
    # the equal-order H derivative does have higher modes (from the face
    # terms), which the mixed system leaves out
    assert np.abs(e[1][:, :, NH:]).max() > 1e-3 * np.abs(e[1]).max()


def test_mixed_central_operator_is_skew():
    verts, tets, eps, mu, rng = _mesh(9, 3)
    K = len(tets)
    O = OracleDG(verts, tets, 3, eps=eps, mu=mu, flux="central", ph=2)
    cE, cH = rng.standard_normal((K, 3, O.N)), rng.standard_normal((K, 3, O.NH))
    dE, dH, _, _ = O.rhs(cE, cH)
    J = O.J[:, None, None]
    a = np.sum(J * eps[:, None, None] * cE * dE)
    b = np.sum(J * mu[:, None, None] * cH * dH)
    assert abs(a + b) < 1e-13 * (abs(a) + abs(b))
    assert abs(a) > 1.0


def _te101_error(n, pe, ph, T=0.2):
    verts, tets = W.kuhn_cube_mesh(n, 0.0, 1.0)
    O = OracleDG(verts, tets, pe, flux="central", ph=ph)
    ones = np.ones(len(tets))
    dt = W.cfl_dt(verts, tets, ones, ones, pe, 0.3)
    ns = int(np.ceil(T / dt))
    dt = T / ns
    cE = O.project(lambda x: W.te101_fields(x, 0.0)[0])
    cH = O.project(lambda x: W.te101_fields(x, 0.0)[1], field="h")
    (e, h, _, _), _ = O.run(cE, cH, dt=dt, nsteps=ns)
    ex = O.project(lambda x: W.te101_fields(x, T)[0])
    hx = O.project(lambda x: W.te101_fields(x, T)[1], field="h")
    return np.sqrt(2.0 * O.energy(e - ex, h - hx))


def test_mixed_cavity_convergence():
    e2, e4 = _te101_error(2, 2, 1), _te101_error(4, 2, 1)
    rate = np.log2(e2 / e4)
    assert rate > 0.8, rate  # central: at least ~ the lower order
    assert e4 < 0.9 * _te101_error(4, 1, 1)  # the richer e space helps
