"""GPU tests of the C ABI's ordering and state contracts.

* A synchronous state write after asynchronous steps on another stream waits
  for those steps: the state read back is exactly the one written, and a step
  from it matches a run that synchronised explicitly.
"""
import numpy as np
import pytest

from tests.gpu_helpers import say, unit_jittered

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_08733_amd import load_library
    load_library()


def _solver(verts, tets, eps, mu, precision="fp64", flux="upwind", dt=1e-3):
    from paper_2002_08733_amd import Solver
    s = Solver(3, precision, flux, dt=dt)
    s.set_mesh(verts, tets)
    s.set_material(eps, mu)
    s.bind_torch_workspace()
    return s


@pytest.mark.parametrize("graph", [True, False])
def test_state_write_waits_for_queued_steps(graph):
    """set_state right after steps queued on a non-blocking torch stream, with
    no synchronisation by the caller (the write goes through the NULL stream)."""
    import torch
    verts, tets, eps, mu = unit_jittered(12, 7)
    say(f"sync test: {len(tets)} tets, graph={graph}")
    rng = np.random.default_rng(3)
    shp = (len(tets), 3, 20)
    E0, H0 = rng.standard_normal(shp), rng.standard_normal(shp)
    E1, H1 = rng.standard_normal(shp), rng.standard_normal(shp)
    s = _solver(verts, tets, eps, mu)
    stream = torch.cuda.Stream()
    s.set_state(E0, H0)
    with torch.cuda.stream(stream):
        if graph:
            s.step_graph(200, 10, stream.cuda_stream)
        else:
            s.step(200, stream.cuda_stream)
    s.set_state(E1, H1)  # no synchronisation in between
    E, H, _ = s.get_state()
    assert np.array_equal(E, E1) and np.array_equal(H, H1)
    with torch.cuda.stream(stream):
        s.step(3, stream.cuda_stream)
    Ea, Ha, _ = s.get_state()
    s.close()
    r = _solver(verts, tets, eps, mu)
    r.set_state(E1, H1)
    r.step(3)
    Eb, Hb, _ = r.get_state()
    r.close()
    assert np.array_equal(Ea, Eb) and np.array_equal(Ha, Hb)


@pytest.mark.parametrize("precision,flux", [("fp64", "upwind"), ("fp32", "central")])
def test_monitor_passes_a_stable_run_unchanged(precision, flux):
    """The energy monitor on a stable source-free run: no error, and the
    state is bitwise the one of the same run without monitor."""
    from paper_2002_08733_amd import Solver
    verts, tets, eps, mu = unit_jittered(5, 17)
    rng = np.random.default_rng(4)
    shp = (len(tets), 3, 20)
    E0, H0 = rng.standard_normal(shp), rng.standard_normal(shp)
    out = []
    for mon in (0, 2, 7):
        s = Solver(3, precision, flux, cfl=0.3, monitor=mon)
        s.set_mesh(verts, tets)
        s.set_material(eps, mu)
        s.bind_torch_workspace()
        s.set_state(E0, H0)
        s.step(30)
        out.append(s.get_state()[:2])
        s.close()
    say(f"monitor stable {precision} {flux}: ok")
    for E, H in out[1:]:
        assert np.array_equal(E, out[0][0]) and np.array_equal(H, out[0][1])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_monitor_reports_an_unstable_run(precision):
    """A step far beyond the stable one (dt = 1 on cells of size 1/4; the
    CFL rule's 0.3 gives 2e-3, and the scheme is still stable at ten times
    that): the energy grows by orders of magnitude within a few steps and
    mdg_step returns MDG_E_UNSTABLE (every launch completes normally)."""
    from paper_2002_08733_amd import Solver
    from paper_2002_08733_amd.mdg import MDG_E_UNSTABLE, MdgError
    verts, tets, eps, mu = unit_jittered(4, 18)
    rng = np.random.default_rng(5)
    shp = (len(tets), 3, 20)
    s = Solver(3, precision, "upwind", dt=1.0, monitor=2)
    s.set_mesh(verts, tets)
    s.set_material(eps, mu)
    s.bind_torch_workspace()
    s.set_state(rng.standard_normal(shp), rng.standard_normal(shp))
    with pytest.raises(MdgError) as e:
        s.step(40)
    say(f"monitor unstable {precision}: {e.value}")
    assert e.value.status == MDG_E_UNSTABLE
    s.close()


def test_monitor_allows_growth_from_a_source():
    """With a dipole the energy grows legitimately: only a non-finite energy
    is an error then."""
    from paper_2002_08733_amd import Solver
    from tests.gpu_helpers import dipole_args
    verts, tets, eps, mu = unit_jittered(4, 19)
    s = Solver(3, "fp64", "upwind", cfl=0.3, monitor=2)
    s.set_mesh(verts, tets)
    s.set_material(eps, mu)
    s.set_dipoles(*dipole_args([(np.array([0.41, 0.52, 0.47]), np.array([0.0, 0.0, 1.0]), (2.0, 1.0))]))
    s.bind_torch_workspace()
    s.step(60)
    assert s.energy() > 0
    s.close()


@pytest.mark.parametrize("precision,flux", [("fp64", "upwind"), ("fp32", "upwind"), ("fp64", "central")])
def test_resume_from_saved_state_is_bitwise(precision, flux):
    """step(2n) is bitwise step(n), get_state, set_state (a fresh handle), step(n):
    the state is the whole of what a source-free RK4 run carries between steps."""
    from paper_2002_08733_amd import Solver
    verts, tets, eps, mu = unit_jittered(6, 23)
    rng = np.random.default_rng(6)
    shp = (len(tets), 3, 20)
    E0, H0 = rng.standard_normal(shp), rng.standard_normal(shp)

    def make():
        s = Solver(3, precision, flux, dt=1e-3)
        s.set_mesh(verts, tets)
        s.set_material(eps, mu)
        s.bind_torch_workspace()
        return s

    a = make()
    a.set_state(E0, H0)
    a.step(24)
    Ea, Ha, ta = a.get_state()
    a.close()
    b = make()
    b.set_state(E0, H0)
    b.step(12)
    E1, H1, t1 = b.get_state()
    b.close()
    c = make()
    c.set_state(E1, H1, t=t1)
    c.step(12)
    Ec, Hc, tc = c.get_state()
    c.close()
    say(f"resume {precision} {flux}: max |diff| {np.abs(Ea - Ec).max():.1e}")
    assert np.array_equal(Ea, Ec) and np.array_equal(Ha, Hc)
    assert abs(ta - tc) < 1e-15
