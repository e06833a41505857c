"""GPU parity at the benchmark sizes and on the edge cases of the decomposition.

* Full-size operator parity, sampled: the 196,608-element jittered cube and the
  663,552-element open-domain PML configuration, evaluated by the library on
  the whole mesh (same tiles and launches as the benchmark), compared with the
  FP64 oracle on a seeded sample of elements (the oracle reads the full state
  for neighbours). Tolerances as in test_gpu_parity.py.
* FP32 state after 1000 RK4 steps of the benchmark workload against the FP64
  state of the library: 1e-5 relative in the energy norm (spec bound;
  the FP64 path itself is oracle-checked in test_gpu_parity.py).
* A mesh whose FP64 state arrays exceed 4 GiB (order 4, 4,374,000 tets,
  7.3 GB per state array): the central scheme's energy identity over every
  element and sampled parity against the oracle.
* Tile-size independence: interior faces resolved in LDS and faces resolved
  through the published halo traces must give the same numbers.
* A mesh made only of PML elements (no non-PML launch), and resetting the
  state between steps (the halo traces of the new state are republished).
"""

import numpy as np
import pytest

import workloads as W
from tests.gpu_helpers import element_bilinear, make_pair, rel_state_err, say, unit_jittered

pytestmark = pytest.mark.gpu

@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_08733_amd import load_library
    load_library()

def _cart(O, u, idx):
    """Covariant coefficients of the elements idx -> Cartesian (A^-T u)."""
    return np.einsum("kji,kjm->kim", O.Ainv[idx], u[idx])

def _sampled_err(O, idx, dE, dH, oE, oH, dP=None, dQ=None, oP=None, oQ=None):
    """Relative energy-norm error on the sampled elements: the larger of the
    error of the whole sample and the per-element maximum
    max_T ||d - o||_T / max_T ||o||_T (one bad element cannot hide)."""
    J, e, m = O.J[idx, None, None], O.eps[idx, None, None], O.mu[idx, None, None]
    cE, cH = _cart(O, dE, idx), _cart(O, dH, idx)
    num = np.sum(J * (e * (cE - oE) ** 2 + m * (cH - oH) ** 2), axis=(1, 2))
    den = np.sum(J * (e * oE ** 2 + m * oH ** 2), axis=(1, 2))
    if dP is not None:
        cP, cQ = _cart(O, dP, idx), _cart(O, dQ, idx)
        num += np.sum(J * ((cP - oP) ** 2 / e + (cQ - oQ) ** 2 / m), axis=(1, 2))
        den += np.sum(J * (oP ** 2 / e + oQ ** 2 / m), axis=(1, 2))
    return float(max(np.sqrt(num.sum() / den.sum()), np.sqrt(num.max() / den.max())))

@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_fullsize_jittered_rhs_sampled(precision, tol):
    w = W.jittered(32, 3, seed=2, flux="upwind")
    say(f"[fullsize rhs] jittered n=32 K={w.nt} p=3 upwind {precision}, 2048 sampled elements")
    s, O = make_pair(w.verts, w.tets, 3, "upwind", precision, w.eps, w.mu)
    rng = np.random.default_rng(21)
    shp = (w.nt, 3, O.N)
    uE, uH = rng.standard_normal(shp), rng.standard_normal(shp)
    dE, dH = s.rhs(uE, uH, t=0.0)
    s.close()
    idx = np.sort(rng.choice(w.nt, size=2048, replace=False))
    oE, oH, _, _ = O.rhs(O.to_cartesian(uE), O.to_cartesian(uH), elems=idx)
    err = _sampled_err(O, idx, dE, dH, oE, oH)
    say(f"  rel err {err:.3e}")
    assert err < tol

@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_fullsize_open_pml_rhs_sampled(precision, tol):
    w = W.open_pml(48, 3)
    pml = np.any(w.omega > 0, axis=1)
    say(f"[fullsize rhs] open PML n=48 K={w.nt} ({pml.sum()} PML) p=3 upwind + dipole {precision}")
    s, O = make_pair(w.verts, w.tets, 3, "upwind", precision, w.eps, w.mu, w.omega, w.dipoles)
    rng = np.random.default_rng(22)
    shp = (w.nt, 3, O.N)
    uE, uH = rng.standard_normal(shp), rng.standard_normal(shp)
    uP, uQ = rng.standard_normal(shp), rng.standard_normal(shp)
    uP[~pml] = 0.0
    uQ[~pml] = 0.0
    t = 1.3  # inside the dipole pulse
    dE, dH, dP, dQ = s.rhs(uE, uH, uP, uQ, t=t, aux=True)
    s.close()
    # half of the sample in the PML, plus the dipole element
    idx = np.unique(np.concatenate([rng.choice(np.flatnonzero(pml), 1024, replace=False),
                                    rng.choice(np.flatnonzero(~pml), 1024, replace=False),
                                    [w.info["dipole_tet"]]]))
    cv = O.to_cartesian
    oE, oH, oP, oQ = O.rhs(cv(uE), cv(uH), cv(uP), cv(uQ), t=t, elems=idx)
    oP[~pml[idx]] = 0.0
    oQ[~pml[idx]] = 0.0
    err = _sampled_err(O, idx, dE, dH, oE, oH, dP, dQ, oP, oQ)
    say(f"  rel err {err:.3e}")
    assert err < tol

def _run_steps(w, precision, steps, dt, tile=0):
    from paper_2002_08733_amd import Solver
    s = Solver(w.p, precision, w.flux, dt=dt, tile=tile)
    s.set_mesh(w.verts, w.tets)
    s.set_material(w.eps, w.mu)
    s.bind_torch_workspace()
    x = s.projection_points(4)
    s.project(4, W.gaussian_curl_e(x, 0.2), None)
    s.step(steps)
    E, H, t = s.get_state()
    return s, E, H

def test_fullsize_fp32_vs_fp64_1000_steps():
    w = W.jittered(32, 3, seed=2, flux="upwind")
    dt = W.cfl_dt(w.verts, w.tets, w.eps, w.mu, w.p, 0.3)
    say(f"[fullsize trajectory] jittered n=32 K={w.nt} p=3 upwind, 1000 RK4 steps, dt={dt:.3e}")
    s32, E32, H32 = _run_steps(w, "fp32", 1000, dt)
    s32.close()
    s64, E64, H64 = _run_steps(w, "fp64", 1000, dt)
    W64 = s64.energy()
    # energy norm of the difference, evaluated by the library's FP64 reduction
    s64.set_state(E32 - E64, H32 - H64)
    Wd = s64.energy()
    s64.close()
    err = float(np.sqrt(Wd / W64))
    # and from the mesh in numpy, globally and per element
    err_el = rel_state_err(w.verts, w.tets, w.eps, w.mu, (E32, H32), (E64, H64))
    say(f"  FP32 vs FP64 rel energy-norm difference {err:.3e} (W = {W64:.6e}); global/per element {err_el:.3e}")
    assert np.isfinite(err) and err < 1e-5
    assert err_el < 1e-5

@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_tile_size_independence(precision):
    w = W.jittered(12, 3, seed=7, flux="upwind")
    dt = W.cfl_dt(w.verts, w.tets, w.eps, w.mu, w.p, 0.3)
    out = {}
    for tile in (32, 64):
        s, E, H = _run_steps(w, precision, 5, dt, tile=tile)
        out[tile] = (E, H, s.query()["tile_size"], s.query()["n_halo"])
        s.close()
    (E1, H1, t1, h1), (E2, H2, t2, h2) = out[32], out[64]
    say(f"[tiles] {precision} K={w.nt}: tile {t1} ({h1} halo faces) vs tile {t2} ({h2} halo faces)")
    assert t1 == 32 and t2 == 64 and h1 != h2
    scale = max(np.abs(E2).max(), np.abs(H2).max())
    d = max(np.abs(E1 - E2).max(), np.abs(H1 - H2).max()) / scale
    say(f"  max difference {d:.3e} of the field scale")
    assert d <= (1e-6 if precision == "fp32" else 1e-14)

def test_all_pml_mesh():
    verts, tets, eps, mu = unit_jittered(4, 31)
    rng = np.random.default_rng(32)
    omega = rng.uniform(0.5, 3.0, (len(tets), 3))
    say(f"[all-PML] K={len(tets)} every element damped, upwind fp64")
    s, O = make_pair(verts, tets, 3, "upwind", "fp64", eps, mu, omega)
    assert s.query()["n_pml"] == len(tets)
    shp = (len(tets), 3, O.N)
    u = [rng.standard_normal(shp) for _ in range(4)]
    dE, dH, dP, dQ = s.rhs(*u, t=0.0, aux=True)
    cv = O.to_cartesian
    oE, oH, oP, oQ = O.rhs(cv(u[0]), cv(u[1]), cv(u[2]), cv(u[3]))
    idx = np.arange(len(tets))
    err = _sampled_err(O, idx, dE, dH, oE, oH, dP, dQ, oP, oQ)
    say(f"  rhs rel err {err:.3e}")
    assert err < 1e-12
    # a few steps against the oracle's RK4
    s.set_state(u[0], u[1], u[2], u[3])
    s.step(3)
    E, H, P, Q, _ = s.get_state(aux=True)
    (cE, cH, cP, cQ), _ = O.run(cv(u[0]), cv(u[1]), cv(u[2]), cv(u[3]), t0=0.0, dt=1e-3, nsteps=3)
    err = _sampled_err(O, idx, E, H, cE, cH, P, Q, cP, cQ)
    say(f"  3 steps rel err {err:.3e}")
    s.close()
    assert err < 1e-12

def test_state_reset_and_rhs_between_steps():
    w = W.jittered(10, 3, seed=8, flux="upwind")
    from paper_2002_08733_amd import Solver

    def solver():
        s = Solver(3, "fp64", "upwind", dt=1e-3)
        s.set_mesh(w.verts, w.tets)
        s.set_material(w.eps, w.mu)
        s.bind_torch_workspace()
        return s

    rng = np.random.default_rng(9)
    shp = (w.nt, 3, 20)
    S1 = (rng.standard_normal(shp), rng.standard_normal(shp))
    S2 = (rng.standard_normal(shp), rng.standard_normal(shp))
    a = solver()
    a.set_state(*S1)
    a.step(3)
    a.set_state(*S2)  # the halo traces of S1's successors must not survive
    a.step(1)
    a.rhs(*S1)  # an operator call between steps leaves the step state alone
    a.step(1)
    Ea, Ha, _ = a.get_state()
    b = solver()
    b.set_state(*S2)
    b.step(2)
    Eb, Hb, _ = b.get_state()
    a.close()
    b.close()
    say(f"[reset] K={w.nt}: max |a-b| = {max(np.abs(Ea - Eb).max(), np.abs(Ha - Hb).max()):.3e}")
    assert np.array_equal(Ea, Eb) and np.array_equal(Ha, Hb)


def test_state_array_beyond_4gib():
    """FP64 at order 4 on 90^3 jittered Kuhn cubes (4,374,000 tets): a state
    array holds 6 x 35 x 8 bytes per element, 7.3 GB, so 41% of the elements
    lie beyond the first 4 GiB of every array. One operator application over
    the whole mesh (central flux, random state, eps and mu): (i) the
    semi-discrete energy identity of the central scheme [KS Sec. III],
    sum_T (eps u.M du + mu f.M df) = 0, checked over all elements against
    sum_T |...|; (ii) parity with the FP64 oracle on 1024 random elements."""
    from oracle import OracleDG
    from paper_2002_08733_amd import Solver
    n, p = 90, 4
    verts, tets = W.kuhn_cube_mesh(n, 0.0, 1.0)
    rng = np.random.default_rng(41)
    verts = W.jitter_interior(verts, 0.0, 1.0, 1.0 / n, 0.1, rng)
    K = len(tets)
    eps = rng.uniform(1.0, 4.0, K)
    mu = rng.uniform(1.0, 2.0, K)
    s = Solver(p, "fp64", "central", dt=1e-4)
    s.set_mesh(verts, tets)
    s.set_material(eps, mu)
    N = s.nmodes
    say(f"[4 GiB] K={K} p={p} fp64 central: state array {6 * N * 8 * K / 1e9:.2f} GB, "
        f"workspace {s.workspace_size() / 1e9:.1f} GB")
    assert 6 * N * 8 * K > 4 << 30
    s.bind_torch_workspace()
    shp = (K, 3, N)
    uE, uH = rng.standard_normal(shp), rng.standard_normal(shp)
    dE, dH = s.rhs(uE, uH, t=0.0)
    s.close()
    b = element_bilinear(verts, tets, eps, mu, (uE, uH), (dE, dH))
    rel = abs(b.sum()) / np.abs(b).sum()
    say(f"  energy identity over all elements: |sum| / sum|.| = {rel:.3e}")
    assert rel < 1e-11
    O = OracleDG(verts, tets, p, eps=eps, mu=mu, flux="central")
    idx = np.sort(rng.choice(K, size=1024, replace=False))
    oE, oH, _, _ = O.rhs(O.to_cartesian(uE), O.to_cartesian(uH), elems=idx)
    err = _sampled_err(O, idx, dE, dH, oE, oH)
    say(f"  sampled rel err vs oracle {err:.3e}")
    assert err < 1e-12
