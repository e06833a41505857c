"""GPU test of the allocation-free probe energy (mdg_probe_energy_noalloc)
against mdg_probe_energy, which allocates its accumulator and probe list:
two calls in a row, the second with fewer probes and steps, each compared with
the allocating entry point on the same state; the state both leave behind
agrees too. Also the size limit and the FP32 path."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_helpers import dipole_args, say, unit_jittered

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_08733_amd import load_library
    load_library()


def _solver(verts, tets, eps, mu, precision):
    from paper_2002_08733_amd import Solver
    s = Solver(3, precision, "upwind", dt=2e-3)
    s.set_mesh(verts, tets)
    s.set_material(eps, mu)
    s.set_dipoles(*dipole_args([(np.array([0.41, 0.52, 0.47]), np.array([0.0, 0.0, 1.0]), (2.0, 1.0))]))
    s.bind_torch_workspace()
    return s


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_probe_energy_matches_allocating_entry(precision):
    verts, tets, eps, mu = unit_jittered(4, 11)
    rng = np.random.default_rng(12)
    shp = (len(tets), 3, 20)
    E0, H0 = 0.1 * rng.standard_normal(shp), 0.1 * rng.standard_normal(shp)
    a = _solver(verts, tets, eps, mu, precision)
    b = _solver(verts, tets, eps, mu, precision)
    calls = [(12, rng.choice(len(tets), 40, replace=False)), (5, rng.choice(len(tets), 7, replace=False))]
    for i, (nsteps, probes) in enumerate(calls):
        say(f"noalloc {precision} call {i}: {nsteps} steps, {len(probes)} probes")
        a.set_state(E0, H0)
        b.set_state(E0, H0)
        Ja = a.probe_energy(nsteps, probes)
        Jb = b.probe_energy_noalloc(nsteps, probes)
        assert Jb == Ja, (i, Ja, Jb)
        assert Ja > 0
        Ea, Ha, ta = a.get_state()
        Eb, Hb, tb = b.get_state()
        assert np.array_equal(Ea, Eb) and np.array_equal(Ha, Hb) and ta == tb
    a.close()
    b.close()


def test_noalloc_probe_energy_rejects_too_many_probes():
    from paper_2002_08733_amd.mdg import MDG_E_ARG, MdgError
    verts, tets, eps, mu = unit_jittered(9, 13)  # 4374 elements
    s = _solver(verts, tets, eps, mu, "fp64")
    with pytest.raises(MdgError) as e:
        s.probe_energy_noalloc(1, np.arange(4097))
    assert e.value.status == MDG_E_ARG
    # the largest allowed list still works and agrees with the allocating call
    probes = np.arange(4096)
    s.set_state(np.zeros((len(tets), 3, 20)), np.zeros((len(tets), 3, 20)))
    J0 = s.probe_energy_noalloc(3, probes)
    s.set_state(np.zeros((len(tets), 3, 20)), np.zeros((len(tets), 3, 20)))
    J1 = s.probe_energy(3, probes)
    assert J0 == J1
    s.close()
