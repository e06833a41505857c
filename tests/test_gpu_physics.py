"""Physics check of the PML on the GPU path (its operator is oracle-checked
in test_gpu_parity.py and test_gpu_fullsize.py): the reflection from the
layer falls monotonically as the layer grows from 1 to 4 elements, measured
as the paper does [KS Sec. V] against a run on a larger domain without PML.

Setup: inner box [-1,1]^3 of 16^3 Kuhn cubes (h = 1/8), p = 3, vacuum, the
z-dipole of the open-domain workload, upwind flux, PML of 1..4 cubes with
the cubic profile (sigma_max = 20). (With the central flux the point source
also excites slowly moving under-resolved modes that linger near it in the
reference run too, which floors this measure near 10%; the upwind flux damps
them, and the reference field leaves the inner box completely.) Reference: [-3,3]^3 with the same
lattice and no PML, whose wall echo cannot reach the inner box before
t = 4. Both meshes share the lattice of the inner box, so its elements and
their covariant frames coincide; the reflection is the largest norm of the
coefficient difference over the inner box at t = 1.25, 2.5, 3.25 and 4,
relative to the largest norm of the reference field there (the outgoing
pulse, at t = 1.25). For the graded profile the continuum estimate is
exp(-2 sigma_max L / 4): 0.7% for 4 layers.

Also: a step far beyond the stability limit is reported as MDG_E_UNSTABLE
by the energy calls.
"""
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


def _run(verts, tets, omega, dip, dt, times, inner_sel, flux="central"):
    from paper_2002_08733_amd import Solver
    s = Solver(3, "fp64", flux, dt=dt)
    s.set_mesh(verts, tets)
    if omega is not None:
        s.set_pml(omega)
    s.set_dipoles(*dip)
    s.bind_torch_workspace()
    out, n = [], 0
    for t in times:
        k = int(round(t / dt))
        s.step(k - n)
        n = k
        E, H, _ = s.get_state()
        out.append((E[inner_sel], H[inner_sel]))
    s.close()
    return out


def _inner(verts, tets):
    """Elements of the inner box and their centroids rounded to the lattice."""
    c = W.tet_centroids(verts, tets)
    sel = np.all(np.abs(c) < 1.0, axis=1)
    key = np.round(c[sel] * 64.0).astype(np.int64)  # centroids sit on a 1/32 lattice
    order = np.lexsort(key.T[::-1])
    return np.flatnonzero(sel)[order], key[order]


def test_pml_reflection_falls_with_thickness():
    times = (1.25, 2.5, 3.25, 4.0)
    ref_verts, ref_tets = W.kuhn_cube_mesh(48, -3.0, 3.0)
    w1 = W.open_pml(18, 3, layers=1)
    d = w1.dipoles[0]
    dip = (d[0][None], d[1][None], np.array([[d[2][0], d[2][1], 5.0 / (2 * np.pi * d[2][1])]]))
    ones = np.ones(len(ref_tets))
    dt = W.cfl_dt(ref_verts, ref_tets, ones, ones, 3, 0.3)
    ref_sel, ref_key = _inner(ref_verts, ref_tets)
    say(f"[PML reflection] reference K={len(ref_tets)} without PML, dt={dt:.3e}, samples at t={times}")
    ref = _run(ref_verts, ref_tets, None, dip, dt, times, ref_sel, "upwind")
    J = np.abs(np.linalg.det(np.stack([ref_verts[ref_tets[ref_sel, i]] - ref_verts[ref_tets[ref_sel, 0]]
                                       for i in (1, 2, 3)], axis=2)))[:, None, None]
    refs = []
    for layers in (1, 2, 3, 4):
        w = W.open_pml(16 + 2 * layers, 3, layers=layers)
        assert np.allclose(w.dipoles[0][0], d[0])
        sel, key = _inner(w.verts, w.tets)
        assert np.array_equal(key, ref_key)
        res = _run(w.verts, w.tets, w.omega, dip, dt, times, sel, "upwind")
        num = max(np.sum(J * ((E - Er) ** 2 + (H - Hr) ** 2)) for (E, H), (Er, Hr) in zip(res, ref))
        den = max(np.sum(J * (Er ** 2 + Hr ** 2)) for Er, Hr in ref)
        refs.append(float(np.sqrt(num / den)))
        say(f"  {layers} layer(s): K={w.nt} ({int(w.omega.any(axis=1).sum())} PML), relative reflection "
            f"{refs[-1]:.3e}")
    assert all(a > 2.0 * b for a, b in zip(refs, refs[1:])), refs
    assert refs[-1] < 0.02


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_unstable_step_is_reported(precision):
    """A time step far beyond the stability limit (RK4: dt rho(L) <= 2 sqrt 2)
    makes the state overflow; mdg_energy and mdg_energy_instances report
    MDG_E_UNSTABLE instead of a number. The condition comes from ordinary
    arithmetic (overflow to inf/nan), nothing faults."""
    from paper_2002_08733_amd import Solver
    from paper_2002_08733_amd.mdg import MDG_E_UNSTABLE, MdgError
    verts, tets = W.kuhn_cube_mesh(2, 0.0, 1.0)
    ones = np.ones(len(tets))
    dt = 60.0 * W.cfl_dt(verts, tets, ones, ones, 3, 0.3)
    s = Solver(3, precision, "upwind", dt=dt)
    s.set_mesh(verts, tets)
    s.bind_torch_workspace()
    rng = np.random.default_rng(31)
    s.set_state(rng.standard_normal((len(tets), 3, 20)), rng.standard_normal((len(tets), 3, 20)))
    W0 = s.energy()
    s.step(200)
    for call in (s.energy, s.energy_instances):
        with pytest.raises(MdgError) as e:
            call()
        assert e.value.status == MDG_E_UNSTABLE
    say(f"[unstable] {precision}: W0 = {W0:.3e}, 200 steps at 60x the CFL step -> MDG_E_UNSTABLE")
    s.close()
