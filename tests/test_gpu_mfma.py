"""GPU tests of the BF16x3 MFMA form of the volume term (mdg_options.mfma):
the reference-curl contraction [KS Sec. III, eq. matrix_free_curl] on the
matrix cores with both operands split exactly into three bfloat16 parts.

* One operator application against the FP64 oracle, orders 1-3, central and
  upwind fluxes, on meshes of several tiles with a ragged last tile, and with
  PML elements and a dipole: the FP32 operator tolerance of the VALU path
  (2e-5 in the energy norm, globally and element by element).
* The same operator with the SIP unknown (central flux, PML) against the VALU
  FP32 path to FP32 rounding.
* Trajectories: 1000 steps of the headline configuration's shape at 8^3 cubes
  against the oracle's golden values are in test_gpu_configs.py.
* Unsupported combinations are refused at creation.
"""
import numpy as np
import pytest

import workloads as W
from oracle import OracleDG
from tests.gpu_helpers import dipole_args, oracle_dipoles, rel_energy_err, say, unit_jittered

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_08733_amd import load_library
    load_library()


def _solver(verts, tets, p, flux, eps, mu, omega=None, dipoles=(), mfma=True, sip_alpha=0.0):
    from paper_2002_08733_amd import Solver
    s = Solver(p, "fp32", flux, dt=1e-3, mfma=mfma, sip_alpha=sip_alpha)
    s.set_mesh(verts, tets)
    s.set_material(eps, mu)
    if omega is not None:
        s.set_pml(omega)
    if dipoles:
        s.set_dipoles(*dipole_args(dipoles))
    s.bind_torch_workspace()
    return s


@pytest.mark.parametrize("flux", ["central", "upwind"])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_mfma_rhs_against_oracle(flux, p):
    verts, tets, eps, mu = unit_jittered(5, 30 + p)  # 750 tets: 11 full tiles and a ragged one
    say(f"[mfma rhs] p={p} {flux}, K={len(tets)}")
    s = _solver(verts, tets, p, flux, eps, mu)
    assert s.query()["tile_size"] == 64
    O = OracleDG(verts, tets, p, eps=eps, mu=mu, flux=flux)
    rng = np.random.default_rng(p)
    shp = (len(tets), 3, O.N)
    uE, uH = rng.standard_normal(shp), rng.standard_normal(shp)
    dE, dH = s.rhs(uE, uH, t=0.2)
    s.close()
    oE, oH, _, _ = O.rhs(O.to_cartesian(uE), O.to_cartesian(uH), t=0.2)
    err = rel_energy_err(O, O.to_cartesian(dE), O.to_cartesian(dH), oE, oH)
    say(f"  rel err {err:.2e}")
    assert err < 2e-5


def test_mfma_rhs_pml_dipole_against_oracle():
    verts, tets, eps, mu = unit_jittered(5, 41)
    c = W.tet_centroids(verts, tets)
    omega = np.zeros((len(tets), 3))
    sel = c[:, 0] > 0.6
    omega[sel, 0] = 4.0
    omega[sel, 2] = 1.5
    dips = [(np.array([0.41, 0.52, 0.47]), np.array([0.2, 0.1, 1.0]), (2.0, 1.0))]
    s = _solver(verts, tets, 3, "upwind", eps, mu, omega=omega, dipoles=dips)
    O = OracleDG(verts, tets, 3, eps=eps, mu=mu, flux="upwind", omega=omega, dipoles=oracle_dipoles(dips))
    rng = np.random.default_rng(9)
    shp = (len(tets), 3, O.N)
    uE, uH, uP, uQ = (rng.standard_normal(shp) for _ in range(4))
    uP[~sel] = 0.0
    uQ[~sel] = 0.0
    dE, dH, dP, dQ = s.rhs(uE, uH, uP, uQ, t=0.7, aux=True)
    s.close()
    cv = O.to_cartesian
    oE, oH, oP, oQ = O.rhs(cv(uE), cv(uH), cv(uP), cv(uQ), t=0.7)
    oP[~sel] = 0.0
    oQ[~sel] = 0.0
    err = rel_energy_err(O, cv(dE), cv(dH), oE, oH, cv(dP), cv(dQ), oP, oQ)
    say(f"[mfma rhs pml dipole] rel err {err:.2e}")
    assert err < 2e-5


def test_mfma_rhs_sip_matches_valu():
    verts, tets, eps, mu = unit_jittered(4, 43)
    c = W.tet_centroids(verts, tets)
    omega = np.zeros((len(tets), 3))
    omega[c[:, 1] > 0.7] = 2.0
    rng = np.random.default_rng(10)
    shp = (len(tets), 3, 20)
    uE, uH = rng.standard_normal(shp), rng.standard_normal(shp)
    uS = rng.standard_normal((len(tets), 4, 2, 10))
    out = []
    for mf in (False, True):
        s = _solver(verts, tets, 3, "central", eps, mu, omega=omega, mfma=mf, sip_alpha=1.0)
        out.append(s.rhs_sip(uE, uH, uS, t=0.1))
        s.close()
    for a, b in zip(out[0], out[1]):
        rel = np.linalg.norm(a - b) / np.linalg.norm(a)
        say(f"[mfma sip] MFMA vs VALU: {rel:.2e}")
        assert rel < 2e-6


def test_mfma_unsupported_combinations_are_refused():
    from paper_2002_08733_amd import Solver
    from paper_2002_08733_amd.mdg import MDG_E_UNSUPPORTED, MdgError
    for kw in (dict(order=3, precision="fp64"), dict(order=4, precision="fp32"),
               dict(order=3, precision="fp32", integrator="leapfrog"), dict(order=3, precision="fp32", tile=32)):
        order = kw.pop("order")
        with pytest.raises(MdgError) as e:
            Solver(order, mfma=True, **kw)
        assert e.value.status == MDG_E_UNSUPPORTED
