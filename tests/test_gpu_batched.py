"""GPU tests of the batched path: independent instances advanced by the same
launches, HIP-graph replay of the step sequence, and the tile autotuner.

* A batch of instances (meshes of 11 to 21 cubes per side) reproduces each
  instance run on its own (same dt, same dipole): the state bit for bit in
  both precisions, the per-instance energy (an FP64 sum whose order differs)
  to rounding.
* One instance of a batch against the FP64 oracle (dipole-driven from zero).
* Graph replay against eager stepping, replayed several times with eager
  work and synchronisations in between; every replay is checked.
* The autotuner returns one of its candidates, with a timing for each, also
  over launch grids.
* Instances with the SIP unknown reproduce their individual runs bit for bit.
* The persistent grid (only the resident workgroups, each looping over its
  tiles) gives the same bits as one workgroup per tile: RK4 with PML elements
  and a dipole, leap-frog halves, and replayed from a HIP graph.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_helpers import oracle_dipoles, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_08733_amd import load_library
    load_library()


def _wave(d):
    f0, bw = d[2]
    return [f0, bw, 5.0 / (2.0 * np.pi * bw)]


def _batch_solver(w, precision, dt, tile=0):
    from paper_2002_08733_amd import Solver
    s = Solver(w.p, precision, w.flux, dt=dt, tile=tile)
    s.set_mesh(w.verts, w.tets)
    s.set_instances(w.info["first"])
    s.set_material(w.eps, w.mu)
    s.set_dipoles(np.array([d[0] for d in w.dipoles]), np.array([d[1] for d in w.dipoles]),
                  np.array([_wave(d) for d in w.dipoles]), instance=[d[3] for d in w.dipoles])
    s.bind_torch_workspace()
    return s


def _instance(w, i):
    """Mesh, material and dipole of instance i as a stand-alone problem."""
    first = w.info["first"]
    tets = w.tets[first[i]:first[i + 1]]
    used = np.unique(tets)
    remap = np.full(w.verts.shape[0], -1, dtype=np.int64)
    remap[used] = np.arange(used.size)
    return w.verts[used], remap[tets], w.eps[first[i]:first[i + 1]], w.mu[first[i]:first[i + 1]], w.dipoles[i]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_matches_individual_runs(precision):
    from paper_2002_08733_amd import Solver
    w = W.batched(4, 3, seed=22, nmin=8, nmax=24)  # sizes 21, 14, 19, 11: 121,170 tets
    dt = W.cfl_dt(w.verts, w.tets, w.eps, w.mu, w.p, 0.3)
    say(f"[batched] {precision}: 4 instances, sizes {list(w.info['sizes'])}, K={w.nt}, dt={dt:.3e}, 30 steps")
    s = _batch_solver(w, precision, dt)
    s.step(30)
    E, H, t = s.get_state()
    Wb = s.energy_instances()
    s.close()
    first = w.info["first"]
    for i in range(4):
        v, tt, eps, mu, d = _instance(w, i)
        r = Solver(3, precision, "upwind", dt=dt)
        r.set_mesh(v, tt)
        r.set_material(eps, mu)
        r.set_dipoles(np.array([d[0]]), np.array([d[1]]), np.array([_wave(d)]))
        r.bind_torch_workspace()
        r.step(30)
        Ei, Hi, ti = r.get_state()
        Wi = r.energy()
        r.close()
        sl = slice(first[i], first[i + 1])
        scale = max(np.abs(Ei).max(), np.abs(Hi).max())
        d_state = max(np.abs(E[sl] - Ei).max(), np.abs(H[sl] - Hi).max()) / scale
        d_energy = abs(Wb[i] - Wi) / Wi
        say(f"  instance {i}: state diff {d_state:.2e}, energy {Wb[i]:.6e} vs {Wi:.6e}")
        assert abs(t - ti) < 1e-15
        # every element's arithmetic is the same in the batch and alone
        assert np.array_equal(E[sl], Ei) and np.array_equal(H[sl], Hi)
        assert d_energy < 1e-13


def test_batch_with_sip_matches_individual_runs():
    """Instances with the SIP unknown (central flux): every instance of the
    batch, h_s included, reproduces its run on its own."""
    from paper_2002_08733_amd import Solver
    w = W.batched(3, 3, seed=23, nmin=2, nmax=4)
    dt = W.cfl_dt(w.verts, w.tets, w.eps, w.mu, w.p, 0.2)

    def make(verts, tets, eps, mu, dips, inst=None, first=None):
        r = Solver(3, "fp64", "central", dt=dt, sip_alpha=1.0)
        r.set_mesh(verts, tets)
        if first is not None:
            r.set_instances(first)
        r.set_material(eps, mu)
        r.set_dipoles(np.array([d[0] for d in dips]), np.array([d[1] for d in dips]),
                      np.array([_wave(d) for d in dips]), instance=inst)
        r.bind_torch_workspace()
        return r

    s = make(w.verts, w.tets, w.eps, w.mu, w.dipoles, [d[3] for d in w.dipoles], w.info["first"])
    s.step(25)
    E, H, _ = s.get_state()
    S = s.get_sip_state()
    s.close()
    first = w.info["first"]
    for i in range(3):
        v, tt, eps, mu, d = _instance(w, i)
        r = make(v, tt, eps, mu, [d])
        r.step(25)
        Ei, Hi, _ = r.get_state()
        Si = r.get_sip_state()
        r.close()
        sl = slice(first[i], first[i + 1])
        diff = max(np.abs(E[sl] - Ei).max(), np.abs(H[sl] - Hi).max(), np.abs(S[sl] - Si).max())
        scale = max(np.abs(Ei).max(), np.abs(Si).max())
        say(f"[batched SIP] instance {i}: max difference {diff / scale:.2e} (|h_s| max {np.abs(Si).max():.2e})")
        assert np.abs(Si).max() > 0 and diff == 0.0


def test_batch_instance_against_oracle():
    from oracle import OracleDG
    from tests.gpu_helpers import rel_energy_err
    w = W.batched(3, 3, seed=17, nmin=2, nmax=4)
    dt = 2e-3
    steps = 12
    say(f"[batched vs oracle] sizes {list(w.info['sizes'])}, fp64, dipole-driven, {steps} steps")
    s = _batch_solver(w, "fp64", dt)
    s.step(steps)
    E, H, _ = s.get_state()
    s.close()
    first = w.info["first"]
    for i in (0, 2):
        v, tt, eps, mu, d = _instance(w, i)
        O = OracleDG(v, tt, 3, eps=eps, mu=mu, flux="upwind", dipoles=oracle_dipoles([d[:3]]))
        z = np.zeros((tt.shape[0], 3, O.N))
        (cE, cH, _, _), _ = O.run(z, z.copy(), t0=0.0, dt=dt, nsteps=steps)
        sl = slice(first[i], first[i + 1])
        err = rel_energy_err(O, O.to_cartesian(E[sl]), O.to_cartesian(H[sl]), cE, cH)
        say(f"  instance {i}: rel err {err:.3e}")
        assert err < 1e-12


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_graph_replay_matches_eager(precision):
    import torch
    w = W.batched(3, 3, seed=19, nmin=3, nmax=6)
    dt = W.cfl_dt(w.verts, w.tets, w.eps, w.mu, w.p, 0.3)
    rng = np.random.default_rng(3)
    shp = (w.nt, 3, 20)
    E0, H0 = rng.standard_normal(shp), rng.standard_normal(shp)
    stream = torch.cuda.Stream()  # default priority
    sp = stream.cuda_stream
    g = _batch_solver(w, precision, dt)
    e = _batch_solver(w, precision, dt)
    for s in (g, e):
        s.set_state(E0, H0, t=0.25)
    say(f"[graph] {precision}: K={w.nt}, graph of 4 steps replayed with eager work in between")
    # 10 steps: two replays and two eager steps; then more replays with
    # eager steps, state reads and energy reductions in between
    plan = [10, 4, 3, 8, 1, 4]
    for k, n in enumerate(plan):
        with torch.cuda.stream(stream):
            g.step_graph(n, 4, sp)
            e.step(n, sp)
        stream.synchronize()
        Eg, Hg, tg = g.get_state()
        Ee, He, te = e.get_state()
        assert tg == te
        same = np.array_equal(Eg, Ee) and np.array_equal(Hg, He)
        say(f"  after {sum(plan[:k + 1])} steps: identical={same}, W={g.energy():.6e}")
        assert same
        if k == 2:  # an eager step on the graph's solver between replays
            g.step(1, sp)
            e.step(1, sp)
            torch.cuda.synchronize()
    g.close()
    e.close()


def test_autotune_tile_returns_a_candidate():
    from paper_2002_08733_amd import Solver
    from paper_2002_08733_amd.autotune import autotune_tile
    w = W.jittered(10, 3, seed=5, flux="upwind")
    dt = W.cfl_dt(w.verts, w.tets, w.eps, w.mu, w.p, 0.3)

    def make(tile):
        s = Solver(3, "fp32", "upwind", dt=dt, tile=tile)
        s.set_mesh(w.verts, w.tets)
        s.set_material(w.eps, w.mu)
        s.bind_torch_workspace()
        return s

    best, times = autotune_tile(make, candidates=(32, 64), steps=5, warmup=2)
    say(f"[autotune] K={w.nt}: {times} -> tile {best}")
    assert best in (32, 64) and set(times) == {32, 64}
    assert all(v > 0 for v in times.values())


def test_autotune_searches_launch_grids():
    from paper_2002_08733_amd import Solver
    from paper_2002_08733_amd.autotune import autotune, launch_candidates
    w = W.jittered(10, 3, seed=5, flux="upwind")
    dt = W.cfl_dt(w.verts, w.tets, w.eps, w.mu, w.p, 0.3)

    def make(tile, launch):
        s = Solver(3, "fp32", "upwind", dt=dt, tile=tile, launch=launch)
        s.set_mesh(w.verts, w.tets)
        s.set_material(w.eps, w.mu)
        s.bind_torch_workspace()
        return s

    cands = launch_candidates("fp32", 3)
    assert len(cands) == 4 and len(launch_candidates("fp64", 3)) == 2
    best, times = autotune(make, cands, steps=5, warmup=2)
    say(f"[autotune] K={w.nt}: {times} -> {best}")
    assert best in cands and set(times) == {"32/per_tile", "64/per_tile", "32/persistent", "64/persistent"}
    assert all(v > 0 for v in times.values())


def _run_launch(w, launch, integrator, steps, graph=False):
    import torch
    from paper_2002_08733_amd import Solver
    cfl = 0.2 if integrator == "leapfrog" else 0.3
    dt = W.cfl_dt(w.verts, w.tets, w.eps, w.mu, w.p, cfl)
    s = Solver(w.p, "fp32", w.flux, dt=dt, integrator=integrator, launch=launch)
    s.set_mesh(w.verts, w.tets)
    s.set_material(w.eps, w.mu)
    if w.omega is not None:
        s.set_pml(w.omega)
    if w.dipoles:
        d = w.dipoles[0]
        s.set_dipoles(d[0][None], d[1][None], np.array([_wave(d)]))
    s.bind_torch_workspace()
    x = s.projection_points(4)
    s.project(4, W.gaussian_curl_e(x, 0.3), None)
    if graph:
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            s.step_graph(steps, 5, stream.cuda_stream)
    else:
        s.step(steps)
    torch.cuda.synchronize()
    E, H, _ = s.get_state()
    q = s.query()
    s.close()
    return E, H, q


@pytest.mark.parametrize("case", ["rk4_pml_dipole", "leapfrog", "rk4_graph"])
def test_persistent_launch_matches_one_workgroup_per_tile(case):
    """More tiles than resident workgroups (256 CUs x 2 for RK4, x 4 for the
    four-lane leap-frog halves), so that the workgroups of the persistent grid
    loop over several tiles."""
    if case == "rk4_pml_dipole":
        w = W.open_pml(28, 3)
    elif case == "leapfrog":
        w = W.jittered(24, 3, seed=3, flux="central")
    else:
        w = W.jittered(24, 3, seed=4, flux="upwind")
    integ = "leapfrog" if case == "leapfrog" else "rk4"
    say(f"[persistent] {case}: K={len(w.tets)}")
    E0, H0, q = _run_launch(w, "per_tile", integ, 10, graph=case == "rk4_graph")
    E1, H1, _ = _run_launch(w, "persistent", integ, 10, graph=case == "rk4_graph")
    assert q["n_tiles"] > 1024
    assert np.abs(E0).max() > 0
    assert np.array_equal(E0, E1) and np.array_equal(H0, H1)
