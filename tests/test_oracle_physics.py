"""Physics pins of the oracle: the TE101 cavity eigenmode of a PEC cube in
closed form (convergence under mesh refinement), energy behaviour of the
central flux (conserved up to the RK4 damping, Sec. III) and of the upwind
flux (non-increasing over two-step windows)."""
import numpy as np
import pytest

import workloads as W
from oracle import OracleDG


def _te101_run(n, p, flux, T):
    verts, tets = W.kuhn_cube_mesh(n, 0.0, 1.0)
    O = OracleDG(verts, tets, p, flux=flux)
    ones = np.ones(len(tets))
    dt = W.cfl_dt(verts, tets, ones, ones, p, 0.3)
    ns = int(np.ceil(T / dt))
    dt = T / ns
    cE = O.project(lambda x: W.te101_fields(x, 0.0)[0])
    cH = O.project(lambda x: W.te101_fields(x, 0.0)[1])
    (e, h, _, _), _ = O.run(cE, cH, dt=dt, nsteps=ns)
    ex = O.project(lambda x: W.te101_fields(x, T)[0])
    hx = O.project(lambda x: W.te101_fields(x, T)[1])
    return np.sqrt(2.0 * O.energy(e - ex, h - hx)), O.energy(cE, cH), O.energy(e, h)


@pytest.mark.parametrize("flux,min_rate", [("upwind", 2.5), ("central", 1.8)])
def test_te101_cavity_convergence(flux, min_rate):
    """p = 2: upwind converges at ~p+1, central at >= ~p (central DG is only
    guaranteed O(h^p) on general meshes)."""
    T = 0.2
    e2, _, _ = _te101_run(2, 2, flux, T)
    e4, _, _ = _te101_run(4, 2, flux, T)
    rate = np.log2(e2 / e4)
    assert rate > min_rate, rate
    assert e4 < 5e-3


def test_central_energy_conserved_upwind_decays():
    verts, tets = W.kuhn_cube_mesh(3, 0.0, 1.0)
    rng = np.random.default_rng(11)
    verts = W.jitter_interior(verts, 0.0, 1.0, 1.0 / 3, 0.1, rng)
    eps = rng.uniform(1.0, 4.0, len(tets))
    ones = np.ones(len(tets))
    dt = W.cfl_dt(verts, tets, eps, ones, 2, 0.3)
    for flux in ("central", "upwind"):
        O = OracleDG(verts, tets, 2, eps=eps, flux=flux)
        cE = O.project(lambda x: W.gaussian_curl_e(x, 0.2, (0.5, 0.5, 0.5)))
        cH = np.zeros_like(cE)
        Ws = [O.energy(cE, cH)]
        s = [cE, cH]
        for _ in range(12):
            (a, b, _, _), _ = O.run(s[0], s[1], dt=dt, nsteps=1)
            s = [a, b]
            Ws.append(O.energy(a, b))
        Ws = np.array(Ws)
        if flux == "central":
            # RK4 damps |R(i y)| = 1 - y^6/72 + ...: tiny and monotone
            assert np.all(np.diff(Ws) <= 1e-14 * Ws[0])
            assert (Ws[0] - Ws[-1]) / Ws[0] < 1e-7
        else:
            assert np.all(Ws[2:] <= Ws[:-2] * (1 + 1e-14))
            assert Ws[-1] < Ws[0]
