"""The benchmark configurations run at their stated accuracy.

* The headline workload's shape at 8^3 cubes (3072 jittered tets, p = 3,
  eps ~ U[1,4], upwind, PEC, Gaussian pulse, RK4 at CFL 0.3) for 1000 steps
  against the FP64 oracle trajectory stored in tests/golden (written by
  tests/golden/make_jittered8_trajectory.py, which calls only the oracle):
  FP64 within 1e-12, FP32 within 1e-5 (relative, energy norm, and per
  element).
* The open-domain configuration at full size (663,552 tets, 279,552 of them
  damped, p = 3, upwind, z-dipole from rest, RK4 at CFL 0.3): FP32 against
  FP64 after its 2000 steps, fields and PML auxiliaries, within 1e-5.
* The batched configuration (64 instances of n_i^3 cubes, n_i ~ U{8..24},
  2,366,874 tets, one launch per stage): FP32 against FP64 after 500 steps,
  within 1e-5 for every instance.
The FP32-against-FP64 comparisons rest on the FP64 path's own oracle parity
(test_gpu_parity.py and the golden trajectory here). Norms are evaluated in
numpy from the mesh (tests.gpu_helpers.element_energy), not by the library.
"""
import os

import numpy as np
import pytest

import workloads as W
from tests.gpu_helpers import dipole_args, element_energy, rel_state_err, say

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "jittered8_p3_upwind_rk4_1000.npz")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_08733_amd import load_library
    load_library()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_jittered8_1000_steps_against_oracle_golden(precision, tol):
    from oracle import OracleDG
    from paper_2002_08733_amd import Solver
    g = np.load(GOLDEN)
    steps, dt = int(g["steps"]), float(g["dt"])
    w = W.jittered(8, 3, seed=2, flux="upwind")
    O = OracleDG(w.verts, w.tets, 3, eps=w.eps, mu=w.mu, flux="upwind")
    cE = O.project(lambda x: W.gaussian_curl_e(x, 0.2))
    cH = np.zeros_like(cE)
    # the stored trajectory starts from this projection
    assert abs(O.energy(cE, cH) / float(g["energy0"]) - 1.0) < 1e-14
    say(f"[golden] jittered n=8 K={w.nt} p=3 upwind {precision}: {steps} RK4 steps, dt={dt:.4e}")
    s = Solver(3, precision, "upwind", dt=dt)
    s.set_mesh(w.verts, w.tets)
    s.set_material(w.eps, w.mu)
    s.bind_torch_workspace()
    s.set_state(O.to_covariant(cE), O.to_covariant(cH))
    s.step(steps)
    E, H, t = s.get_state()
    s.close()
    assert abs(t - steps * dt) < 1e-12 * steps * dt
    ref = (O.to_covariant(g["cE"]), O.to_covariant(g["cH"]))
    err = rel_state_err(w.verts, w.tets, w.eps, w.mu, (E, H), ref)
    say(f"  rel err vs oracle after {steps} steps: {err:.3e}")
    assert err < tol


def _run(w, precision, steps, dt, dipoles=True, instances=None):
    from paper_2002_08733_amd import Solver
    s = Solver(w.p, precision, w.flux, dt=dt)
    s.set_mesh(w.verts, w.tets)
    if instances is not None:
        s.set_instances(instances)
    s.set_material(w.eps, w.mu)
    if w.omega is not None:
        s.set_pml(w.omega)
    if dipoles and w.dipoles:
        pos, dr, wave = dipole_args(w.dipoles)
        inst = [d[3] for d in w.dipoles] if instances is not None else None
        s.set_dipoles(pos, dr, wave, instance=inst)
    s.bind_torch_workspace()
    return s


def test_open_pml_fp32_vs_fp64_2000_steps():
    w = W.open_pml(48, 3)
    dt = W.cfl_dt(w.verts, w.tets, w.eps, w.mu, w.p, 0.3)
    steps = w.steps
    say(f"[open PML] K={w.nt} ({int(np.any(w.omega > 0, axis=1).sum())} PML) p=3 upwind, dipole from rest, "
        f"{steps} RK4 steps, dt={dt:.3e}")
    out = {}
    for prec in ("fp32", "fp64"):
        s = _run(w, prec, steps, dt)
        s.step(steps)
        out[prec] = s.get_state(aux=True)[:4]
        Wl = s.energy()
        s.close()
        say(f"  {prec}: library energy {Wl:.6e}")
    a, b = out["fp32"], out["fp64"]
    Wb = element_energy(w.verts, w.tets, w.eps, w.mu, *b)
    assert np.isfinite(Wb).all() and Wb.sum() > 0
    err = rel_state_err(w.verts, w.tets, w.eps, w.mu, a, b)
    say(f"  FP32 vs FP64 rel difference (fields and auxiliaries, global and per element): {err:.3e}")
    assert err < 1e-5


def test_batched_64_instances_fp32_vs_fp64_500_steps():
    w = W.batched(64, 3, seed=4)
    dt = W.cfl_dt(w.verts, w.tets, w.eps, w.mu, w.p, 0.3)
    first = w.info["first"]
    steps = w.steps
    say(f"[batched] {len(first) - 1} instances, K={w.nt} p=3 upwind + dipoles, {steps} RK4 steps, dt={dt:.3e}")
    out = {}
    for prec in ("fp32", "fp64"):
        s = _run(w, prec, steps, dt, instances=first)
        s.step(steps)
        out[prec] = s.get_state()[:2]
        s.close()
    a, b = out["fp32"], out["fp64"]
    d = element_energy(w.verts, w.tets, w.eps, w.mu, a[0] - b[0], a[1] - b[1])
    r = element_energy(w.verts, w.tets, w.eps, w.mu, *b)
    worst = 0.0
    for i in range(len(first) - 1):
        sl = slice(first[i], first[i + 1])
        assert r[sl].sum() > 0
        e = max(np.sqrt(d[sl].sum() / r[sl].sum()), np.sqrt(d[sl].max() / r[sl].max()))
        worst = max(worst, e)
        assert e < 1e-5, (i, e)
    say(f"  worst instance FP32 vs FP64 rel difference (global and per element): {worst:.3e}")
