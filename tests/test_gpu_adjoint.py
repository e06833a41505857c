"""GPU tests of the adjoint (gradient of the probe energy w.r.t. every
element's permittivity): against the oracle's matrix adjoint on a tiny mesh,
against central finite differences of the library's own objective on 16
elements (both also with PML elements, and the finite differences with mixed
orders, the upwind flux and the SIP unknown), independence of the checkpoint
interval, and the autograd entry."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_08733_amd import load_library
    load_library()


def _solver(verts, tets, p, eps, dt, precision="fp64", dip=None, omega=None, mixed=False, flux="central",
            mu=None, sip_alpha=0.0):
    from paper_2002_08733_amd import Solver
    s = Solver(p, precision, flux, dt=dt, mixed=mixed, sip_alpha=sip_alpha)
    s.set_mesh(verts, tets)
    s.set_material(eps, mu)
    if omega is not None:
        s.set_pml(omega)
    if dip is not None:
        s.set_dipoles(*dip)
    s.bind_torch_workspace()
    return s


def _tiny():
    verts, tets = W.kuhn_cube_mesh(2, 0.0, 1.0)
    rng = np.random.default_rng(41)
    verts = W.jitter_interior(verts, 0.0, 1.0, 0.5, 0.1, rng)
    return verts, tets


def _tiny_omega(rng):
    omega = np.zeros((48, 3))
    sel = rng.random(48) < 0.5
    omega[sel] = rng.uniform(1.0, 8.0, (sel.sum(), 3))
    omega[sel & (rng.random(48) < 0.4), 2] = 0.0
    return omega


def _one_cube():
    """One cube of 6 tets with every vertex moved (12 PEC faces, 6 interior)."""
    verts, tets = W.kuhn_cube_mesh(1, 0.0, 1.0)
    return verts + 0.06 * np.random.default_rng(48).standard_normal(verts.shape), tets


# FP64 against the exact oracle adjoint (closed form for the central flux,
# complex-step impedance derivative for the upwind flux) to 1e-12; FP32 state
# with FP64 reductions to 2e-4
@pytest.mark.parametrize("precision,tol,pml,flux,sip,mixed", [
    ("fp64", 1e-12, False, "central", False, False), ("fp32", 2e-4, False, "central", False, False),
    ("fp64", 1e-12, True, "central", False, False), ("fp32", 2e-4, True, "central", False, False),
    ("fp64", 1e-12, False, "upwind", False, False), ("fp64", 1e-12, True, "upwind", False, False),
    ("fp32", 2e-4, True, "upwind", False, False),
    ("fp64", 1e-12, False, "central", True, False), ("fp64", 1e-12, True, "central", True, False),
    ("fp32", 2e-4, True, "central", True, False), ("fp64", 1e-12, True, "central", True, True)])
def test_adjoint_matches_oracle_adjoint(precision, tol, pml, flux, sip, mixed):
    from oracle import OracleDG
    from oracle.adjoint import adjoint_gradient
    from oracle.sip import SipDG
    rng = np.random.default_rng(42)
    if sip:  # the SIP oracle assembles its operator column by column: one cube
        verts, tets = _one_cube()
        K, probes, pos = len(tets), np.array([1, 4]), np.array([0.45, 0.5, 0.55])
        omega = None
        if pml:
            omega = np.zeros((K, 3))
            sel = np.array([True, False, True, False, False, True])
            omega[sel] = rng.uniform(1.0, 6.0, (sel.sum(), 3))
    else:
        verts, tets = _tiny()
        K, probes, pos = 48, np.array([3, 17, 40]), np.array([0.4, 0.45, 0.55])
        omega = _tiny_omega(rng) if pml else None
    eps = rng.uniform(1.0, 4.0, K)
    dr = np.array([0.3, 0.2, 1.0])
    mu = np.linspace(1.0, 2.0, K)
    pe = 2 if mixed else 1  # order of e; h at order 1
    O = OracleDG(verts, tets, pe, eps=eps, mu=mu, flux=flux, omega=omega, ph=1,
                 dipoles=[(pos, dr, lambda t: W.dipole_waveform(t, 2.0, 1.0))])
    cE0 = 0.3 * rng.standard_normal((K, 3, O.N))
    cH0 = 0.3 * rng.standard_normal((K, 3, O.NH))
    dt, nsteps = (0.005, 6) if sip else (0.01, 8)
    Jo, go = adjoint_gradient(O, cE0, cH0, dt, nsteps, probes, sip=SipDG(O, 1.0) if sip else None)
    dip = (pos[None], dr[None], np.array([[2.0, 1.0, 5.0 / (2 * np.pi)]]))
    s = _solver(verts, tets, 1, eps, dt, precision, dip, omega, flux=flux, mu=mu, mixed=mixed,
                sip_alpha=1.0 if sip else 0.0)
    s.set_state(O.to_covariant(cE0), O.to_covariant(cH0))
    J, g = s.adjoint_probe_energy(nsteps, 3, probes)
    s.close()
    eJ = abs(J - Jo) / abs(Jo)
    eg = np.abs(g - go).max() / np.abs(go).max()
    say(f"[adjoint vs oracle] {precision} {flux} pml={pml} sip={sip} mixed={mixed}: J {J:.12e} vs {Jo:.12e} "
        f"({eJ:.2e}), grad max rel {eg:.2e}")
    assert eJ < tol and eg < tol


def _medium(n=4, p=2, seed=51):
    w = W.jittered(n, p, seed=seed, flux="central")
    rng = np.random.default_rng(seed + 1)
    E0 = 0.2 * rng.standard_normal((w.nt, 3, W.nmodes(p)))
    H0 = 0.2 * rng.standard_normal((w.nt, 3, W.nmodes(p)))
    dip = (np.array([[0.1, -0.2, 0.15]]), np.array([[0.0, 0.0, 1.0]]), np.array([[2.0, 1.0, 5.0 / (2 * np.pi)]]))
    return w, E0, H0, dip


@pytest.mark.parametrize("case", ["plain", "pml", "mixed_pml", "upwind_pml", "sip_pml", "mixed_sip_pml"])
def test_adjoint_matches_finite_differences_on_16_elements(case):
    w, E0, H0, dip = _medium()
    omega, mixed = None, case.startswith("mixed")
    sip = 1.0 if "sip" in case else 0.0  # the SIP unknown starts at zero
    flux = "upwind" if case.startswith("upwind") else "central"
    if case != "plain":
        # a damped slab (x > 0.4), one axis undamped on part of it
        c = W.tet_centroids(w.verts, w.tets)
        omega = np.zeros((w.nt, 3))
        sel = c[:, 0] > 0.4
        omega[sel, 0] = 6.0 * ((c[sel, 0] - 0.4) / 0.6) ** 2
        omega[sel, 1] = 2.0
        omega[sel & (c[:, 2] > 0.0), 2] = 1.5
    if mixed:  # e at order 2, h at order 1
        H0 = H0[:, :, :W.nmodes(w.p - 1)]
    dt, nsteps, every = 2e-3, 60, 16
    probes = np.array([5, 77, 150, 222, 301, 333, 360, 383])
    p = w.p - 1 if mixed else w.p

    def make(eps):
        s = _solver(w.verts, w.tets, p, eps, dt, dip=dip, omega=omega, mixed=mixed, flux=flux, sip_alpha=sip)
        s.set_state(E0, H0)
        return s

    s = make(w.eps)
    J, g = s.adjoint_probe_energy(nsteps, every, probes)
    npml = s.query()["n_pml"]
    s.close()
    rng = np.random.default_rng(7)
    elems = np.unique(np.concatenate([probes, rng.choice(w.nt, 8, replace=False)]))[:16]
    if omega is not None:  # half of the checked elements damped
        damped = np.flatnonzero(omega.any(axis=1))
        elems = np.unique(np.concatenate([elems[:8], rng.choice(damped, 8, replace=False)]))
    say(f"[adjoint FD] {case}: K={w.nt} ({npml} PML) p={w.p}, {nsteps} steps, checkpoint every {every}, J={J:.10e}")
    worst = 0.0
    for T in elems:
        h = 1e-6 * w.eps[T]
        Jpm = []
        for sgn in (1, -1):
            e = w.eps.copy()
            e[T] += sgn * h
            s = make(e)
            Jpm.append(s.adjoint_probe_energy(nsteps, nsteps, probes)[0])
            s.close()
        fd = (Jpm[0] - Jpm[1]) / (2 * h)
        # FD round-off is ~1e-16 |J| / h in absolute terms, so elements whose
        # gradient is tiny are held to the scale of the whole gradient
        bound = 1e-5 * abs(fd) + 1e-7 * np.abs(g).max()
        ratio = abs(g[T] - fd) / bound
        worst = max(worst, ratio)
        say(f"  element {T}: adjoint {g[T]:+.8e}  fd {fd:+.8e}  |diff|/bound {ratio:.2f}")
    assert worst <= 1.0


def test_adjoint_checkpoint_interval_independence():
    w, E0, H0, dip = _medium(5, 3, 61)
    dt, nsteps = 1e-3, 40
    probes = np.array([0, 100, 500, 749])
    out = {}
    for every in (1, 7, 40):
        s = _solver(w.verts, w.tets, w.p, w.eps, dt, dip=dip)
        s.set_state(E0, H0)
        out[every] = s.adjoint_probe_energy(nsteps, every, probes)
        E, H, t = s.get_state()
        assert abs(t - nsteps * dt) < 1e-15
        s.close()
    say(f"[adjoint checkpoints] J = {[out[e][0] for e in out]}")
    for every in (7, 40):
        assert out[every][0] == out[1][0]
        assert np.array_equal(out[every][1], out[1][1])


def test_adjoint_fullsize_pml_against_finite_differences():
    """The adjoint configuration at full size, FP64: 24^3 cubes x 6 = 82,944
    tets with a PML 3 cubes thick (57.8% of the elements), p=3, central
    flux, z-dipole, 8 probes, 2000 steps, checkpoint every 100; central
    differences (delta = 1e-6 eps) of the forward objective on the 8 probe
    elements and 8 random ones (seed 5)."""
    from paper_2002_08733_amd import Solver
    w = W.adjoint_pml()
    dt = W.cfl_dt(w.verts, w.tets, w.eps, w.mu, w.p, 0.3)
    probes = w.info["probes"]
    d = w.dipoles[0]
    dip = (d[0][None], d[1][None], np.array([[d[2][0], d[2][1], 5.0 / (2 * np.pi * d[2][1])]]))
    nsteps = 2000

    def make(eps):
        s = Solver(3, "fp64", "central", dt=dt)
        s.set_mesh(w.verts, w.tets)
        s.set_material(eps, w.mu)
        s.set_pml(w.omega)
        s.set_dipoles(*dip)
        s.bind_torch_workspace()
        return s

    s = make(w.eps)
    say(f"[adjoint full size] K={w.nt} ({s.query()['n_pml']} PML), {nsteps} steps, checkpoint every 100")
    J, g = s.adjoint_probe_energy(nsteps, 100, probes)
    s.close()
    s = make(w.eps)
    Jf = s.probe_energy(nsteps, probes)
    s.close()
    say(f"  J = {J:.12e} (forward only {Jf:.12e}), |grad| max {np.abs(g).max():.3e}")
    assert J == Jf
    rng = np.random.default_rng(5)
    elems = np.concatenate([probes, rng.choice(w.nt, 8, replace=False)])
    worst = 0.0
    for T in elems:
        h = 1e-6 * w.eps[T]
        Jpm = []
        for sgn in (1, -1):
            e = w.eps.copy()
            e[T] += sgn * h
            s = make(e)
            Jpm.append(s.probe_energy(nsteps, probes))
            s.close()
        fd = (Jpm[0] - Jpm[1]) / (2 * h)
        bound = 1e-5 * abs(fd) + 1e-7 * np.abs(g).max()
        ratio = abs(g[T] - fd) / bound
        worst = max(worst, ratio)
        say(f"  element {T} ({'PML' if w.omega[T].any() else 'inner'}): adjoint {g[T]:+.8e}  fd {fd:+.8e}  "
            f"|diff|/bound {ratio:.2f}")
    assert worst <= 1.0


@pytest.mark.parametrize("case", ["plain", "pml", "upwind_pml", "sip_pml"])
def test_autograd_function(case):
    import torch
    from paper_2002_08733_amd.autograd import ProbeEnergyProblem
    w, E0, H0, dip = _medium()
    probes = np.array([5, 222])
    omega = None
    pml = case != "plain"
    if pml:
        c = W.tet_centroids(w.verts, w.tets)
        omega = np.zeros((w.nt, 3))
        omega[c[:, 0] > 0.4] = 3.0
    prob = ProbeEnergyProblem(w.verts, w.tets, w.p, E0, H0, 2e-3, 20, 5, probes, dipoles=dip, omega=omega,
                              flux="upwind" if case.startswith("upwind") else "central",
                              sip_alpha=1.0 if case.startswith("sip") else 0.0)
    eps = torch.tensor(w.eps, dtype=torch.float64, requires_grad=True)
    J = prob(eps)
    (gt,) = torch.autograd.grad(3.0 * J, eps)
    Jd, gd = prob.run(w.eps)
    say(f"[autograd] {case}: J={J.item():.10e}")
    assert J.item() == Jd
    assert np.array_equal(gt.numpy(), 3.0 * gd)
    # without a gradient request only the forward steps run: the same J
    with torch.no_grad():
        assert prob(eps).item() == Jd
    assert prob(torch.tensor(w.eps, dtype=torch.float64)).item() == Jd
    # the same objective through the library directly, finite differences on one element
    T = 222
    h = 1e-6 * w.eps[T]
    e1, e2 = w.eps.copy(), w.eps.copy()
    e1[T] += h
    e2[T] -= h
    fd = (prob.run(e1)[0] - prob.run(e2)[0]) / (2 * h)
    prob.close()
    assert abs(gd[T] - fd) <= 1e-5 * abs(fd) + 1e-7 * np.abs(gd).max()
