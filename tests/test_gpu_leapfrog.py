"""GPU tests of the leap-frog integrator (the paper's time scheme [KS Sec. V])
against the oracle's staggered scheme (oracle/leapfrog.py).

* FP64 and FP32 trajectories driven by a dipole (sources at the half step)
  from a random staggered state, on a mesh of several tiles with a ragged
  tail, against leapfrog_run.
* The staggered energy 1/2 (e^n, eps e^n) + 1/2 (h^{n-1/2}, mu h^{n+1/2}) of
  the library's own states is conserved to round-off over 300 steps.
* PML elements, damping terms by the trapezoid rule, against
  leapfrog_pml_run (FP64 and FP32).
* Tile-size independence and HIP-graph replay of leap-frog steps.
* The adjoint (an RK4 construction) refuses a leap-frog solver.
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


def _solver(verts, tets, eps, mu, precision, dt, omega=None, dipoles=(), tile=0):
    from paper_2002_08733_amd import Solver
    s = Solver(3, precision, "central", dt=dt, tile=tile, integrator="leapfrog")
    s.set_mesh(verts, tets)
    s.set_material(eps, mu)
    if omega is not None:
        s.set_pml(omega)
    if dipoles:
        s.set_dipoles(*dipole_args(dipoles))
    s.bind_torch_workspace()
    return s


def _dipole():
    return [(np.array([0.47, 0.52, 0.49]), np.array([0.3, -0.2, 0.9]), (2.0, 1.0))]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_leapfrog_trajectory_against_oracle(precision, tol):
    from oracle import OracleDG
    from oracle.leapfrog import leapfrog_run
    verts, tets, eps, mu = unit_jittered(5, 41)
    K = len(tets)
    dt = W.cfl_dt(verts, tets, eps, mu, 3, 0.2)
    dip = _dipole()
    rng = np.random.default_rng(42)
    E0, H0 = 0.05 * rng.standard_normal((K, 3, 20)), 0.05 * rng.standard_normal((K, 3, 20))
    t0, steps = 0.6, 25  # inside the dipole pulse
    say(f"[leapfrog] {precision}: K={K} p=3 central + dipole, dt={dt:.3e}, {steps} steps from t={t0}")
    s = _solver(verts, tets, eps, mu, precision, dt, dipoles=dip)
    s.set_state(E0, H0, t=t0)
    s.step(steps)
    E, H, t = s.get_state()
    q = s.query()
    s.close()
    assert q["n_tiles"] > 1
    O = OracleDG(verts, tets, 3, eps=eps, mu=mu, flux="central", dipoles=oracle_dipoles(dip))
    cE, cH, to = leapfrog_run(O, O.to_cartesian(E0), O.to_cartesian(H0), t0, dt, steps)
    err = rel_energy_err(O, O.to_cartesian(E), O.to_cartesian(H), cE, cH)
    say(f"  rel err {err:.3e}, time {t:.6f} vs {to:.6f}")
    assert abs(t - to) < 1e-12
    assert err < tol


def test_leapfrog_staggered_energy_conserved():
    from oracle import OracleDG
    from oracle.leapfrog import staggered_energy
    verts, tets, eps, mu = unit_jittered(5, 43)
    K = len(tets)
    dt = W.cfl_dt(verts, tets, eps, mu, 3, 0.2)
    rng = np.random.default_rng(44)
    s = _solver(verts, tets, eps, mu, "fp64", dt)
    s.set_state(rng.standard_normal((K, 3, 20)), rng.standard_normal((K, 3, 20)))
    O = OracleDG(verts, tets, 3, eps=eps, mu=mu, flux="central")
    cv = O.to_cartesian

    def w_after_next_step():
        _, Hp, _ = s.get_state()
        s.step(1)
        E, H, _ = s.get_state()
        return staggered_energy(O, cv(E), cv(Hp), cv(H))

    W1 = w_after_next_step()
    s.step(297)
    W299 = w_after_next_step()
    s.close()
    say(f"[leapfrog energy] K={K}: W^1 = {W1:.15e}, W^299 = {W299:.15e}, rel change {(W299 - W1) / W1:.2e}")
    assert abs(W299 - W1) < 1e-12 * W1


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_leapfrog_trapezoid_pml_against_oracle(precision, tol):
    from oracle import OracleDG
    from oracle.leapfrog import leapfrog_pml_run
    verts, tets, eps, mu = unit_jittered(5, 45)
    K = len(tets)
    rng = np.random.default_rng(46)
    omega = np.zeros((K, 3))
    c = W.tet_centroids(verts, tets)
    pml = c[:, 0] > 0.55  # a slab of damped elements, some with one axis undamped
    omega[pml] = rng.uniform(1.0, 6.0, (pml.sum(), 3))
    omega[pml & (c[:, 1] < 0.3), 2] = 0.0
    dt = W.cfl_dt(verts, tets, eps, mu, 3, 0.2)
    shp = (K, 3, 20)
    E0, H0 = rng.standard_normal(shp), rng.standard_normal(shp)
    P0, Q0 = rng.standard_normal(shp), rng.standard_normal(shp)
    P0[~pml] = 0.0
    Q0[~pml] = 0.0
    dip = _dipole()
    steps = 20
    say(f"[leapfrog PML] {precision}: K={K} ({pml.sum()} PML) central + dipole, {steps} steps")
    s = _solver(verts, tets, eps, mu, precision, dt, omega=omega, dipoles=dip)
    assert s.query()["n_pml"] == pml.sum()
    s.set_state(E0, H0, P0, Q0, t=0.6)
    s.step(steps)
    E, H, P, Q, _ = s.get_state(aux=True)
    s.close()
    O = OracleDG(verts, tets, 3, eps=eps, mu=mu, flux="central", omega=omega, dipoles=oracle_dipoles(dip))
    cv = O.to_cartesian
    cE, cH, cP, cQ, _ = leapfrog_pml_run(O, cv(E0), cv(H0), cv(P0), cv(Q0), 0.6, dt, steps)
    err = rel_energy_err(O, cv(E), cv(H), cE, cH, cv(P), cv(Q), cP, cQ)
    say(f"  rel err {err:.3e}")
    assert err < tol


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_leapfrog_tile_independence_and_graph(precision):
    import torch
    w = W.jittered(10, 3, seed=47, flux="central")
    dt = W.cfl_dt(w.verts, w.tets, w.eps, w.mu, w.p, 0.2)
    rng = np.random.default_rng(48)
    shp = (w.nt, 3, 20)
    E0, H0 = rng.standard_normal(shp), rng.standard_normal(shp)
    out = {}
    for tile in (32, 64):
        s = _solver(w.verts, w.tets, w.eps, w.mu, precision, dt, tile=tile)
        s.set_state(E0, H0)
        s.step(12)
        out[tile] = s.get_state()[:2] + (s.query()["n_halo"],)
        s.close()
    (E1, H1, h1), (E2, H2, h2) = out[32], out[64]
    scale = max(np.abs(E2).max(), np.abs(H2).max())
    d = max(np.abs(E1 - E2).max(), np.abs(H1 - H2).max()) / scale
    say(f"[leapfrog tiles] {precision} K={w.nt}: halo faces {h1} vs {h2}, max difference {d:.3e}")
    assert h1 != h2 and d <= (1e-6 if precision == "fp32" else 1e-14)
    # graph replay against eager stepping, several replays with eager work between
    stream = torch.cuda.Stream()  # default priority
    sp = stream.cuda_stream
    g = _solver(w.verts, w.tets, w.eps, w.mu, precision, dt)
    e = _solver(w.verts, w.tets, w.eps, w.mu, precision, dt)
    for x in (g, e):
        x.set_state(E0, H0, t=0.1)
    for n in (9, 4, 7):
        with torch.cuda.stream(stream):
            g.step_graph(n, 4, sp)
            e.step(n, sp)
        stream.synchronize()
        Eg, Hg, tg = g.get_state()
        Ee, He, te = e.get_state()
        say(f"  graph vs eager after {n} more steps: identical={np.array_equal(Eg, Ee) and np.array_equal(Hg, He)}")
        assert tg == te and np.array_equal(Eg, Ee) and np.array_equal(Hg, He)
        g.energy()
    g.close()
    e.close()


def test_adjoint_refuses_leapfrog():
    from paper_2002_08733_amd.mdg import MDG_E_UNSUPPORTED, MdgError
    verts, tets, eps, mu = unit_jittered(2, 49)
    s = _solver(verts, tets, eps, mu, "fp64", 1e-3)
    with pytest.raises(MdgError) as ei:
        s.adjoint_probe_energy(4, 2, np.array([0, 1]))
    s.close()
    assert ei.value.status == MDG_E_UNSUPPORTED
