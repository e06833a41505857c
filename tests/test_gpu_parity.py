"""GPU parity: libmdg (HIP kernels on gfx950, called through the C ABI) against
the FP64 oracle on the same seeded inputs, compared in the oracle's Cartesian
frame with the relative energy norm.

Tolerances. FP64 operator: the kernel and the oracle evaluate the same
polynomial operator with different (but exact) quadrature and summation
orders; their difference is rounding, amplified by the operator norm
~ (p+1)^2 / h relative to the coefficients: 1e-12 relative is ~1e3 ulps.
FP64 trajectories: 1e-12 relative after the run (spec bound).
FP32 operator: unit roundoff 6e-8 times the same amplification: 2e-5.
"""
import numpy as np
import pytest

import workloads as W
from oracle import OracleDG
from tests.gpu_helpers import dipole_args, make_pair, oracle_dipoles, rel_energy_err, say, unit_jittered

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_08733_amd import load_library
    load_library()


def _rhs_case(verts, tets, p, flux, eps, mu, precision="fp64", omega=None, dipoles=(), t=0.3, seed=0):
    s, O = make_pair(verts, tets, p, flux, precision, eps, mu, omega, dipoles)
    rng = np.random.default_rng(seed)
    shp = (len(tets), 3, O.N)
    uE, uH = rng.standard_normal(shp), rng.standard_normal(shp)
    if omega is not None:
        uP, uQ = rng.standard_normal(shp), rng.standard_normal(shp)
        pml = np.any(omega > 0, axis=1)
        uP[~pml] = 0.0
        uQ[~pml] = 0.0
        dE, dH, dP, dQ = s.rhs(uE, uH, uP, uQ, t=t, aux=True)
        oE, oH, oP, oQ = O.rhs(O.to_cartesian(uE), O.to_cartesian(uH), O.to_cartesian(uP),
                               O.to_cartesian(uQ), t=t)
        oP[~pml] = 0.0
        oQ[~pml] = 0.0
        err = rel_energy_err(O, O.to_cartesian(dE), O.to_cartesian(dH), oE, oH,
                             O.to_cartesian(dP), O.to_cartesian(dQ), oP, oQ)
    else:
        dE, dH = s.rhs(uE, uH, t=t)
        oE, oH, _, _ = O.rhs(O.to_cartesian(uE), O.to_cartesian(uH), t=t)
        err = rel_energy_err(O, O.to_cartesian(dE), O.to_cartesian(dH), oE, oH)
    s.close()
    return err


@pytest.mark.parametrize("flux", ["central", "upwind"])
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_rhs_parity_fp64(flux, p):
    say(f"[rhs fp64] flux={flux} p={p} mesh=unit n=3 jittered")
    verts, tets, eps, mu = unit_jittered(3, 10 + p)
    err = _rhs_case(verts, tets, p, flux, eps, mu)
    say(f"  rel err {err:.3e}")
    assert err < 1e-12


@pytest.mark.parametrize("flux", ["central", "upwind"])
def test_rhs_parity_many_tiles_fp64(flux):
    say(f"[rhs fp64 multi-tile] flux={flux} n=6 p=3")
    verts, tets, eps, mu = unit_jittered(6, 3, -1.0, 1.0)
    err = _rhs_case(verts, tets, 3, flux, eps, mu)
    say(f"  rel err {err:.3e}")
    assert err < 1e-12


@pytest.mark.parametrize("flux", ["central", "upwind"])
def test_rhs_parity_fp32(flux):
    say(f"[rhs fp32] flux={flux} n=4 p=3")
    verts, tets, eps, mu = unit_jittered(4, 5, -1.0, 1.0)
    err = _rhs_case(verts, tets, 3, flux, eps, mu, precision="fp32")
    say(f"  rel err {err:.3e}")
    assert err < 2e-5


@pytest.mark.parametrize("flux", ["central", "upwind"])
@pytest.mark.parametrize("p", [1, 2, 4])
def test_rhs_parity_fp32_other_orders(flux, p):
    say(f"[rhs fp32] flux={flux} p={p} mesh=unit n=3 jittered")
    verts, tets, eps, mu = unit_jittered(3, 30 + p)
    err = _rhs_case(verts, tets, p, flux, eps, mu, precision="fp32")
    say(f"  rel err {err:.3e}")
    assert err < 2e-5


@pytest.mark.parametrize("flux", ["central", "upwind"])
def test_rhs_parity_pml_fp64(flux):
    say(f"[rhs pml fp64] flux={flux}")
    w = W.open_pml(n=12, p=2, layers=3, flux=flux)
    err = _rhs_case(w.verts, w.tets, 2, flux, w.eps, w.mu, omega=w.omega, dipoles=w.dipoles, t=0.31)
    say(f"  rel err {err:.3e}")
    assert err < 1e-12


def test_rhs_parity_dipole_fp64():
    say("[rhs dipole fp64]")
    verts, tets, eps, mu = unit_jittered(3, 8)
    dips = [(np.array([0.37, 0.52, 0.44]), np.array([0.2, -0.4, 0.9]), (2.0, 1.0)),
            (np.array([0.81, 0.13, 0.67]), np.array([0.0, 0.0, 1.0]), (1.5, 0.7))]
    err = _rhs_case(verts, tets, 3, "upwind", eps, mu, dipoles=dips, t=0.37)
    say(f"  rel err {err:.3e}")
    assert err < 1e-12


def test_single_element_and_scrambled_order():
    """Edge cases: one tetrahedron (all faces PEC); element order and vertex
    order inside tets scrambled (results follow the caller's order)."""
    say("[edge] single tet, scrambled order")
    verts = np.array([[0, 0, 0], [1.1, 0.1, 0], [0.2, 0.9, 0.1], [0.1, 0.2, 1.3]])
    tets = np.array([[2, 0, 3, 1]])
    err = _rhs_case(verts, tets, 3, "upwind", np.array([2.0]), np.array([1.5]))
    say(f"  single rel err {err:.3e}")
    assert err < 1e-12
    verts, tets, eps, mu = unit_jittered(3, 9)
    rng = np.random.default_rng(2)
    perm = rng.permutation(len(tets))
    tets = np.array([row[rng.permutation(4)] for row in tets[perm]])
    err = _rhs_case(verts, tets, 2, "upwind", eps[perm], mu[perm])
    say(f"  scrambled rel err {err:.3e}")
    assert err < 1e-12


def test_state_roundtrip_and_energy():
    say("[state/energy]")
    verts, tets, eps, mu = unit_jittered(3, 4)
    s, O = make_pair(verts, tets, 3, "upwind", "fp64", eps, mu)
    rng = np.random.default_rng(1)
    shp = (len(tets), 3, O.N)
    uE, uH = rng.standard_normal(shp), rng.standard_normal(shp)
    s.set_state(uE, uH, t=0.25)
    E, H, t = s.get_state()
    assert t == 0.25
    np.testing.assert_array_equal(E, uE)
    np.testing.assert_array_equal(H, uH)
    w = s.energy()
    wo = O.energy(O.to_cartesian(uE), O.to_cartesian(uH))
    say(f"  energy {w} oracle {wo}")
    assert abs(w - wo) < 1e-12 * wo
    s.close()


def test_projection_matches_oracle():
    """Library projection of a polynomial field (exact for both quadratures)."""
    say("[projection]")
    verts, tets, eps, mu = unit_jittered(2, 6)
    s, O = make_pair(verts, tets, 3, "central", "fp64", eps, mu)

    def f(x):
        X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
        return np.stack([X * Y * Z, X ** 3 - Y, Z * Z + X], -1)

    x = s.projection_points(6)
    s.project(6, f(x), None)
    E, H, _ = s.get_state()
    cE = O.project(f)
    err = np.abs(O.to_cartesian(E) - cE).max() / np.abs(cE).max()
    say(f"  max rel diff {err:.3e}")
    assert err < 1e-13
    assert np.abs(H).max() == 0.0
    s.close()


def test_cavity_te101_trajectory():
    """PEC unit cube, 4^3 x 6 tets, p=2, vacuum, TE101 initial field, central
    flux, RK4 at CFL 0.3, 100 steps, FP64: GPU vs oracle <= 1e-12 relative."""
    say("[cavity] 384 tets p=2 central 100 steps fp64")
    w = W.cavity(4, 2)
    ones = np.ones(w.nt)
    dt = W.cfl_dt(w.verts, w.tets, ones, ones, 2, 0.3)
    s, O = make_pair(w.verts, w.tets, 2, "central", "fp64", w.eps, w.mu, dt=dt)
    cE = O.project(lambda x: W.te101_fields(x, 0.0)[0])
    cH = O.project(lambda x: W.te101_fields(x, 0.0)[1])
    s.set_state(O.to_covariant(cE), O.to_covariant(cH))
    s.step(100)
    E, H, t = s.get_state()
    (oE, oH, _, _), to = O.run(cE, cH, dt=dt, nsteps=100)
    err = rel_energy_err(O, O.to_cartesian(E), O.to_cartesian(H), oE, oH)
    say(f"  t={t:.6f} oracle t={to:.6f} rel err {err:.3e}")
    assert abs(t - to) < 1e-12
    assert err < 1e-12
    # the discrete solution approximates the eigenmode (sanity, not parity)
    ex = O.project(lambda x: W.te101_fields(x, t)[0])
    hx = O.project(lambda x: W.te101_fields(x, t)[1])
    assert rel_energy_err(O, O.to_cartesian(E), O.to_cartesian(H), ex, hx, elementwise=False) < 2e-2
    s.close()


def test_jittered_upwind_trajectory_fp64_and_fp32():
    """The jittered-cube workload at reduced size (8^3 x 6 tets, p=3, eps in
    [1,4], upwind, Gaussian pulse) for 20 RK4 steps: FP64 GPU vs oracle
    <= 1e-12; FP32 GPU vs FP64 GPU within 1e-5 (error of the FP32 state)."""
    say("[jittered] n=8 p=3 upwind 20 steps")
    w = W.jittered(8, 3, seed=2)
    dt = W.cfl_dt(w.verts, w.tets, w.eps, w.mu, 3, 0.3)
    s, O = make_pair(w.verts, w.tets, 3, "upwind", "fp64", w.eps, w.mu, dt=dt)
    cE = O.project(lambda x: W.gaussian_curl_e(x, 0.2))
    cH = np.zeros_like(cE)
    s.set_state(O.to_covariant(cE), O.to_covariant(cH))
    s.step(20)
    E, H, _ = s.get_state()
    (oE, oH, _, _), _ = O.run(cE, cH, dt=dt, nsteps=20)
    err = rel_energy_err(O, O.to_cartesian(E), O.to_cartesian(H), oE, oH)
    say(f"  fp64 rel err {err:.3e}")
    assert err < 1e-12
    s.close()
    s32, _ = make_pair(w.verts, w.tets, 3, "upwind", "fp32", w.eps, w.mu, dt=dt)
    s32.set_state(O.to_covariant(cE), O.to_covariant(cH))
    s32.step(20)
    E32, H32, _ = s32.get_state()
    err32 = rel_energy_err(O, O.to_cartesian(E32), O.to_cartesian(H32), O.to_cartesian(E), O.to_cartesian(H))
    say(f"  fp32 vs fp64 rel err {err32:.3e}")
    assert err32 < 1e-5
    s32.close()


def test_pml_dipole_trajectory_fp64():
    """Open-domain workload at reduced size (12^3 cubes, PML 3 layers,
    z-dipole), 20 steps FP64 GPU vs oracle, auxiliaries included."""
    say("[pml] n=12 p=2 upwind dipole 20 steps")
    w = W.open_pml(n=12, p=2, layers=3)
    dt = W.cfl_dt(w.verts, w.tets, w.eps, w.mu, 2, 0.3)
    s, O = make_pair(w.verts, w.tets, 2, "upwind", "fp64", w.eps, w.mu, w.omega, w.dipoles, dt=dt)
    z = np.zeros((w.nt, 3, O.N))
    s.set_state(z, z, z, z, t=0.0)
    s.step(20)
    E, H, P, Q, t = s.get_state(aux=True)
    (oE, oH, oP, oQ), _ = O.run(z, z, z.copy(), z.copy(), dt=dt, nsteps=20)
    pml = np.any(w.omega > 0, axis=1)
    oP[~pml] = 0.0
    oQ[~pml] = 0.0
    err = rel_energy_err(O, O.to_cartesian(E), O.to_cartesian(H), oE, oH,
                         O.to_cartesian(P), O.to_cartesian(Q), oP, oQ)
    say(f"  rel err {err:.3e}")
    assert err < 1e-12
    s.close()


def test_determinism():
    say("[determinism]")
    w = W.jittered(6, 3, seed=2)
    outs = []
    for _ in range(2):
        from paper_2002_08733_amd import Solver
        s = Solver(3, "fp32", "upwind", dt=1e-3)
        s.set_mesh(w.verts, w.tets)
        s.set_material(w.eps, w.mu)
        s.bind_torch_workspace()
        rng = np.random.default_rng(3)
        shp = (w.nt, 3, 20)
        s.set_state(rng.standard_normal(shp), rng.standard_normal(shp))
        s.step(5)
        outs.append(s.get_state()[:2])
        s.close()
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])


def test_1000_steps_against_oracle_fp64_and_fp32():
    """1000 RK4 steps against the FP64 oracle on a small mesh (48 jittered
    tets, p=3, upwind, PML on half of the elements, a dipole, 32-element tiles
    so that the halo path and a ragged tail are in it): FP64 within 1e-12 and
    FP32 within 1e-5 relative in the energy norm, the bounds the method is
    held to after 1000 steps."""
    from paper_2002_08733_amd import Solver
    verts, tets, eps, mu = unit_jittered(2, 71)
    K = len(tets)
    rng = np.random.default_rng(72)
    omega = np.zeros((K, 3))
    sel = rng.random(K) < 0.5
    omega[sel] = rng.uniform(0.5, 4.0, (sel.sum(), 3))
    dip = [(np.array([0.45, 0.55, 0.5]), np.array([0.2, -0.3, 0.9]), (2.0, 1.0))]
    dt = W.cfl_dt(verts, tets, eps, mu, 3, 0.3)
    steps = 1000
    O = OracleDG(verts, tets, 3, eps=eps, mu=mu, flux="upwind", omega=omega, dipoles=oracle_dipoles(dip))
    cE = O.project(lambda x: W.gaussian_curl_e(x, 0.3, (0.5, 0.5, 0.5)))
    cH = np.zeros_like(cE)
    say(f"[1000 steps] K={K} ({sel.sum()} PML) p=3 upwind + dipole, dt={dt:.3e}: oracle trajectory")
    (oE, oH, oP, oQ), _ = O.run(cE, cH, dt=dt, nsteps=steps)
    for precision, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        s = Solver(3, precision, "upwind", dt=dt, tile=32)
        s.set_mesh(verts, tets)
        s.set_material(eps, mu)
        s.set_pml(omega)
        s.set_dipoles(*dipole_args(dip))
        s.bind_torch_workspace()
        assert s.query()["n_tiles"] >= 2
        s.set_state(O.to_covariant(cE), O.to_covariant(cH))
        s.step(steps)
        E, H, P, Q, _ = s.get_state(aux=True)
        s.close()
        cv = O.to_cartesian
        err = rel_energy_err(O, cv(E), cv(H), oE, oH, cv(P), cv(Q), oP, oQ)
        say(f"  {precision}: rel err after {steps} steps {err:.3e} (bound {tol:.0e})")
        assert err < tol
