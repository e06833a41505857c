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
