"""GPU parity of the SIP surface unknown [KS Sec. III, eqs. jmp_var_def,
1st_weak_equation, weak_penalty] against the oracle (oracle/sip.py).

* One operator application (mdg_rhs_sip; equal and mixed orders) with PML
  elements, a dipole and uneven materials.
* RK4 trajectories (FP64, FP32) from random e, h, h_s with PML elements, a
  dipole and uneven materials, on meshes of several tiles with a ragged tail;
  FP64 RK4 at orders 1, 2 and 4 as well.
* The paper's own scheme: leap-frog with h_s beside h, PML damping by the
  trapezoid rule, a dipole (FP64, FP32).
* The two copies of each interior face's h_s stay equal to round-off, the
  staggered energy with the h_s term is conserved over 200 leap-frog steps,
  and the result does not depend on the tile size.
* Full size (the benchmark's SIP configuration): staggered energy with the
  h_s term conserved and both copies of every face equal.
* Mixed orders (e at p+1, h and h_s at p) with RK4, and the paper's whole
  scheme: mixed orders, leap-frog, trapezoid PML, a dipole and h_s.
* set_state clears h_s; set/get round trip; HIP-graph replay of SIP steps
  equals eager stepping (several replays with eager work between them).

Errors are relative, in the energy norm of the whole state (e, h, h_s, p, q)
of the oracle.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_helpers import dipole_args, oracle_dipoles, say, unit_jittered

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_08733_amd import load_library
    load_library()


def _pair(verts, tets, p, precision, eps, mu, alpha0, dt, omega=None, dipoles=(), integrator="rk4", tile=0,
          mixed=False):
    """Library solver and oracle; with mixed, e at order p + 1 and h, h_s at p."""
    from oracle import OracleDG
    from oracle.sip import SipDG
    from paper_2002_08733_amd import Solver
    s = Solver(p, precision, "central", dt=dt, integrator=integrator, sip_alpha=alpha0, tile=tile, mixed=mixed)
    s.set_mesh(verts, tets)
    s.set_material(eps, mu)
    if omega is not None:
        s.set_pml(omega)
    if dipoles:
        s.set_dipoles(*dipole_args(dipoles))
    s.bind_torch_workspace()
    O = OracleDG(verts, tets, p + (1 if mixed else 0), eps=eps, mu=mu, flux="central", omega=omega,
                 dipoles=oracle_dipoles(dipoles), ph=p)
    S = SipDG(O, alpha0)
    assert (s.nmodes, s.nmodes_h, s.nfacemodes) == (O.N, O.NH, S.NF)
    return s, S


def _pml_omega(verts, tets, rng):
    c = W.tet_centroids(verts, tets)
    omega = np.zeros((len(tets), 3))
    sel = c[:, 0] > 0.6
    omega[sel] = rng.uniform(1.0, 5.0, (sel.sum(), 3))
    omega[sel & (c[:, 1] < 0.3), 2] = 0.0
    return omega, sel


def _dip():
    return [(np.array([0.45, 0.5, 0.52]), np.array([0.1, 0.3, 0.95]), (2.0, 1.0))]


def _rel(S, got, want):
    """Relative error in the oracle's energy norm; got/want = (e, h, h_s[faces], p, q)."""
    d = [None if a is None else a - b for a, b in zip(got, want)]
    num = S.energy(d[0], d[1], d[2])
    den = S.energy(want[0], want[1], want[2])
    if want[3] is not None:
        O = S.O
        J = O.J[:, None, None]
        for a, b, m in ((d[3], want[3], O.eps), (d[4], want[4], O.mu)):
            num += 0.5 * np.sum(J * a * a / m[:, None, None])
            den += 0.5 * np.sum(J * b * b / m[:, None, None])
    return float(np.sqrt(num / den))


def _random_state(S, rng, pml=None):
    O = S.O
    K, N, NH = O.K, O.N, O.NH
    E, H = rng.standard_normal((K, 3, N)), rng.standard_normal((K, 3, NH))
    Sf = rng.standard_normal((S.nfaces, 2, S.NF))
    P = Q = None
    if pml is not None:
        P, Q = rng.standard_normal((K, 3, N)), rng.standard_normal((K, 3, NH))
        P[~pml] = 0.0
        Q[~pml] = 0.0
    return E, H, Sf, P, Q


@pytest.mark.parametrize("precision,tol,mixed", [("fp64", 1e-12, False), ("fp32", 2e-5, False),
                                                 ("fp64", 1e-12, True)])
def test_sip_operator_parity(precision, tol, mixed):
    """One operator application (mdg_rhs_sip) against the oracle: PML
    elements, a dipole at its time, uneven materials, several tiles."""
    verts, tets, eps, mu = unit_jittered(4, 94)
    rng = np.random.default_rng(95)
    omega, pml = _pml_omega(verts, tets, rng)
    s, S = _pair(verts, tets, 2 if mixed else 3, precision, eps, mu, 1.3, 1e-3, omega, _dip(), mixed=mixed)
    E, H, Sf, P, Q = _random_state(S, rng, pml)
    O = S.O
    cov, cv = O.to_covariant, O.to_cartesian
    t = 0.8
    dE, dH, dS, dP, dQ = s.rhs_sip(cov(E), cov(H), S.to_sides(Sf), cov(P), cov(Q), t=t, aux=True)
    s.close()
    oE, oH, oS, oP, oQ = S.rhs(E, H, Sf, P, Q, t=t)
    oP[~pml] = 0.0
    oQ[~pml] = 0.0
    err = _rel(S, (cv(dE), cv(dH), S.from_sides(dS), cv(dP), cv(dQ)), (oE, oH, oS, oP, oQ))
    other = np.stack([dS[o // 4, o % 4] for (_, _, o) in S.sides if o >= 0])
    first = np.stack([dS[k, f] for (k, f, o) in S.sides if o >= 0])
    dcopy = np.abs(other - first).max() / np.abs(first).max()
    say(f"[SIP rhs] {'e3/h2' if mixed else 'p=3'} {precision}: K={O.K} ({pml.sum()} PML): rel err {err:.3e}, "
        f"copies {dcopy:.1e}")
    assert err < tol and dcopy < (1e-13 if precision == "fp64" else 1e-5)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_sip_rk4_trajectory_with_pml_and_dipole(precision, tol):
    verts, tets, eps, mu = unit_jittered(4, 71)
    rng = np.random.default_rng(72)
    omega, pml = _pml_omega(verts, tets, rng)
    dt = W.cfl_dt(verts, tets, eps, mu, 3, 0.1)
    s, S = _pair(verts, tets, 3, precision, eps, mu, 1.5, dt, omega, _dip())
    E, H, Sf, P, Q = _random_state(S, rng, pml)
    O = S.O
    cov = O.to_covariant
    s.set_state(cov(E), cov(H), cov(P), cov(Q), t=0.5)
    s.set_sip_state(S.to_sides(Sf))
    q = s.query()
    say(f"[SIP RK4] p=3 {precision}: K={O.K} ({pml.sum()} PML), {S.nfaces} faces, {q['n_tiles']} tiles, dt={dt:.3e}")
    s.step(6)
    gE, gH, gP, gQ, t = s.get_state(aux=True)
    gS = s.get_sip_state()
    s.close()
    (oE, oH, oS, oP, oQ), to = S.rk4_run(E, H, Sf, P, Q, t0=0.5, dt=dt, nsteps=6)
    cv = O.to_cartesian
    err = _rel(S, (cv(gE), cv(gH), S.from_sides(gS), cv(gP), cv(gQ)), (oE, oH, oS, oP, oQ))
    # the other copy of every interior face
    other = np.stack([gS[o // 4, o % 4] for (_, _, o) in S.sides if o >= 0])
    first = np.stack([gS[k, f] for (k, f, o) in S.sides if o >= 0])
    dcopy = np.abs(other - first).max() / np.abs(first).max()
    say(f"  rel err {err:.3e}, copies of interior faces differ by {dcopy:.2e}")
    assert abs(t - to) < 1e-12 and err < tol
    assert dcopy < (1e-13 if precision == "fp64" else 1e-5)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_sip_leapfrog_trapezoid_pml(precision, tol):
    verts, tets, eps, mu = unit_jittered(5, 73)
    rng = np.random.default_rng(74)
    omega, pml = _pml_omega(verts, tets, rng)
    dt = W.cfl_dt(verts, tets, eps, mu, 3, 0.05)
    s, S = _pair(verts, tets, 3, precision, eps, mu, 1.0, dt, omega, _dip(), integrator="leapfrog")
    E, H, Sf, P, Q = _random_state(S, rng, pml)
    O = S.O
    cov = O.to_covariant
    s.set_state(cov(E), cov(H), cov(P), cov(Q), t=0.6)
    s.set_sip_state(S.to_sides(Sf))
    s.step(15)
    gE, gH, gP, gQ, _ = s.get_state(aux=True)
    gS = s.get_sip_state()
    s.close()
    oE, oH, oS, oP, oQ, _ = S.leapfrog_run(E, H, Sf, P, Q, t0=0.6, dt=dt, nsteps=15)
    cv = O.to_cartesian
    err = _rel(S, (cv(gE), cv(gH), S.from_sides(gS), cv(gP), cv(gQ)), (oE, oH, oS, oP, oQ))
    say(f"[SIP leap-frog] p=3 {precision}: K={O.K} ({pml.sum()} PML), 15 steps: rel err {err:.3e}")
    assert err < tol


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_sip_mixed_orders_the_papers_scheme(precision, tol):
    """e at order 3, h and h_s at order 2, leap-frog with the PML damping by
    the trapezoid rule, a dipole and the SIP unknown: the paper's scheme."""
    verts, tets, eps, mu = unit_jittered(5, 82)
    rng = np.random.default_rng(83)
    omega, pml = _pml_omega(verts, tets, rng)
    dt = W.cfl_dt(verts, tets, eps, mu, 3, 0.05)
    s, S = _pair(verts, tets, 2, precision, eps, mu, 1.0, dt, omega, _dip(), integrator="leapfrog", mixed=True)
    E, H, Sf, P, Q = _random_state(S, rng, pml)
    O = S.O
    cov = O.to_covariant
    s.set_state(cov(E), cov(H), cov(P), cov(Q), t=0.6)
    s.set_sip_state(S.to_sides(Sf))
    s.step(12)
    gE, gH, gP, gQ, _ = s.get_state(aux=True)
    gS = s.get_sip_state()
    s.close()
    oE, oH, oS, oP, oQ, _ = S.leapfrog_run(E, H, Sf, P, Q, t0=0.6, dt=dt, nsteps=12)
    cv = O.to_cartesian
    err = _rel(S, (cv(gE), cv(gH), S.from_sides(gS), cv(gP), cv(gQ)), (oE, oH, oS, oP, oQ))
    say(f"[SIP mixed leap-frog] e3/h2/h_s2 {precision}: K={O.K} ({pml.sum()} PML), 12 steps: rel err {err:.3e}")
    assert err < tol


def test_sip_mixed_rk4():
    verts, tets, eps, mu = unit_jittered(4, 84)
    rng = np.random.default_rng(85)
    dt = W.cfl_dt(verts, tets, eps, mu, 3, 0.1)
    s, S = _pair(verts, tets, 2, "fp64", eps, mu, 2.0, dt, mixed=True)
    E, H, Sf, _, _ = _random_state(S, rng)
    O = S.O
    s.set_state(O.to_covariant(E), O.to_covariant(H), t=0.1)
    s.set_sip_state(S.to_sides(Sf))
    s.step(6)
    gE, gH, _ = s.get_state()
    gS = s.get_sip_state()
    s.close()
    (oE, oH, oS, _, _), _ = S.rk4_run(E, H, Sf, t0=0.1, dt=dt, nsteps=6)
    cv = O.to_cartesian
    err = _rel(S, (cv(gE), cv(gH), S.from_sides(gS), None, None), (oE, oH, oS, None, None))
    say(f"[SIP mixed RK4] e3/h2/h_s2 fp64: rel err {err:.3e}")
    assert err < 1e-12


def test_sip_leapfrog_staggered_energy_and_tiles():
    verts, tets, eps, mu = unit_jittered(5, 75)
    dt = W.cfl_dt(verts, tets, eps, mu, 2, 0.05)
    rng = np.random.default_rng(76)
    out = {}
    for tile in (32, 64):
        s, S = _pair(verts, tets, 2, "fp64", eps, mu, 2.0, dt, integrator="leapfrog", tile=tile)
        O = S.O
        E, H, Sf, _, _ = _random_state(S, np.random.default_rng(77))
        s.set_state(O.to_covariant(E), O.to_covariant(H))
        s.set_sip_state(S.to_sides(Sf))
        cv = O.to_cartesian

        def w_next():
            _, Hp, _ = s.get_state()
            Sp = S.from_sides(s.get_sip_state())
            s.step(1)
            e, h, _ = s.get_state()
            return S.staggered_energy(cv(e), cv(Hp), cv(h), Sp, S.from_sides(s.get_sip_state()))

        W1 = w_next()
        s.step(200)
        W2 = w_next()
        out[tile] = s.get_state()[:2] + (s.get_sip_state(), s.query()["n_halo"])
        s.close()
        say(f"[SIP leap-frog energy] tile {tile}: W {W1:.15e} -> {W2:.15e} ({(W2 - W1) / W1:.1e})")
        assert abs(W2 - W1) < 1e-12 * W1
    (E1, H1, S1, h1), (E2, H2, S2, h2) = out[32], out[64]
    d = max(np.abs(E1 - E2).max(), np.abs(H1 - H2).max(), np.abs(S1 - S2).max())
    say(f"  tiles 32 vs 64: halo faces {h1} vs {h2}, max difference {d:.2e}")
    assert h1 != h2 and d < 1e-11 * max(np.abs(E2).max(), np.abs(S2).max())


def test_sip_state_roundtrip_and_reset():
    verts, tets, eps, mu = unit_jittered(3, 78)
    s, S = _pair(verts, tets, 2, "fp64", eps, mu, 1.0, 1e-3)
    rng = np.random.default_rng(79)
    K = len(tets)
    Ss = rng.standard_normal((K, 4, 2, S.NF))
    E = rng.standard_normal((K, 3, 10))
    s.set_state(E, E)
    s.set_sip_state(Ss)
    assert np.array_equal(s.get_sip_state(), Ss)
    s.set_state(E, E)  # a new state starts with h_s = 0
    assert not s.get_sip_state().any()
    s.close()


def test_sip_graph_replay_matches_eager():
    import torch
    verts, tets, eps, mu = unit_jittered(4, 80)
    dt = W.cfl_dt(verts, tets, eps, mu, 3, 0.1)
    rng = np.random.default_rng(81)
    stream = torch.cuda.Stream()  # default priority
    sp = stream.cuda_stream
    pair = [_pair(verts, tets, 3, "fp32", eps, mu, 1.0, dt) for _ in range(2)]
    g, e = pair[0][0], pair[1][0]
    S = pair[0][1]
    E, H, Sf, _, _ = _random_state(S, rng)
    for x in (g, e):
        x.set_state(S.O.to_covariant(E), S.O.to_covariant(H), t=0.2)
        x.set_sip_state(S.to_sides(Sf))
    for n in (9, 4, 7):
        with torch.cuda.stream(stream):
            g.step_graph(n, 4, sp)
            e.step(n, sp)
        stream.synchronize()
        same = np.array_equal(g.get_sip_state(), e.get_sip_state()) and all(
            np.array_equal(a, b) for a, b in zip(g.get_state(), e.get_state()))
        say(f"[SIP graph] after {n} more steps: graph == eager: {same}")
        assert same
        g.energy()
    g.close()
    e.close()


@pytest.mark.parametrize("p", [1, 2, 4])
def test_sip_rk4_other_orders(p):
    verts, tets, eps, mu = unit_jittered(3, 86 + p)
    rng = np.random.default_rng(90 + p)
    dt = W.cfl_dt(verts, tets, eps, mu, p, 0.1)
    s, S = _pair(verts, tets, p, "fp64", eps, mu, 1.0, dt)
    E, H, Sf, _, _ = _random_state(S, rng)
    O = S.O
    s.set_state(O.to_covariant(E), O.to_covariant(H))
    s.set_sip_state(S.to_sides(Sf))
    s.step(4)
    gE, gH, _ = s.get_state()
    gS = s.get_sip_state()
    s.close()
    (oE, oH, oS, _, _), _ = S.rk4_run(E, H, Sf, dt=dt, nsteps=4)
    cv = O.to_cartesian
    err = _rel(S, (cv(gE), cv(gH), S.from_sides(gS), None, None), (oE, oH, oS, None, None))
    say(f"[SIP RK4] p={p} fp64: K={O.K}, NF={S.NF}: rel err {err:.3e}")
    assert err < 1e-12


# ------------------------------------------------------------ full size
_FACE_VERTS = ((1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2))


def _fullsize_tables(verts, tets, mu, p, alpha0):
    """Closed-form quantities of the staggered energy on every element side
    (vectorised for the full mesh; the face mass (mu_F/alpha_F) sqrt(det g)
    g^-1 (x) I is pinned against the oracle's quadrature in
    test_oracle_sip.py): the side weight c = w (mu_F/alpha_F) |t1 x t2| with
    w = 1/2 on interior faces (both copies) and 1 on PEC faces, g^-1, the
    other side (element * 4 + face, or -1), and A^-1, J per element."""
    T = np.sort(np.asarray(tets, dtype=np.int64), axis=1)
    X = np.asarray(verts, dtype=np.float64)[T]
    A = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    J = np.abs(np.linalg.det(A))
    K = len(T)
    keys = np.stack([T[:, list(fv)] for fv in _FACE_VERTS], axis=1).reshape(-1, 3)
    _, inv = np.unique(keys, axis=0, return_inverse=True)
    inv = inv.ravel()
    order = np.argsort(inv, kind="stable")
    srt = inv[order]
    pair = np.nonzero(srt[1:] == srt[:-1])[0]
    other = -np.ones(4 * K, dtype=np.int64)
    other[order[pair]] = order[pair + 1]
    other[order[pair + 1]] = order[pair]
    other = other.reshape(K, 4)
    t1 = np.stack([X[:, fv[1]] - X[:, fv[0]] for fv in _FACE_VERTS], axis=1)
    t2 = np.stack([X[:, fv[2]] - X[:, fv[0]] for fv in _FACE_VERTS], axis=1)
    cr = np.linalg.norm(np.cross(t1, t2), axis=-1)
    has = other >= 0
    kn = np.where(has, other // 4, np.arange(K)[:, None])
    alpha = alpha0 * (p + 1) * (p + 3) / 3.0 * 0.5 * cr / np.minimum(J[:, None], J[kn]) * 6.0
    muF = 0.5 * (mu[:, None] + mu[kn])
    c = np.where(has, 0.5, 1.0) * muF / alpha * cr
    g11, g12, g22 = (t1 * t1).sum(-1), (t1 * t2).sum(-1), (t2 * t2).sum(-1)
    det = g11 * g22 - g12 * g12
    ginv = np.stack([np.stack([g22, -g12], -1), np.stack([-g12, g11], -1)], -2) / det[..., None, None]
    return c, ginv, other, np.linalg.inv(A), J


def _fullsize_staggered_energy(tab, eps, mu, E, Hp, Hn, Sp, Sn):
    c, ginv, _, Ainv, J = tab
    cart = lambda u: np.einsum("kji,kjm->kim", Ainv, u)  # noqa: E731
    cE, cHp, cHn = cart(E), cart(Hp), cart(Hn)
    We = 0.5 * np.sum(J * eps * np.sum(cE * cE, axis=(1, 2)))
    Wh = 0.5 * np.sum(J * mu * np.sum(cHp * cHn, axis=(1, 2)))
    Ws = 0.5 * np.sum(c * np.einsum("kfam,kfab,kfbm->kf", Sp, ginv, Sn))
    return We + Wh + Ws, Ws


def test_sip_fullsize_leapfrog_properties():
    """The benchmark's SIP configuration (196,608-element jittered cube, p=3,
    central flux, leap-frog at CFL 0.2, alpha0 = 1, same launches), FP64:
    the staggered energy with the h_s term is conserved, and the two copies
    of every interior face's h_s agree (properties that hold at any size)."""
    from paper_2002_08733_amd import Solver
    w = W.jittered(32, 3, seed=2, flux="central")
    dt = W.cfl_dt(w.verts, w.tets, w.eps, w.mu, 3, 0.2)
    s = Solver(3, "fp64", "central", dt=dt, integrator="leapfrog", sip_alpha=1.0)
    s.set_mesh(w.verts, w.tets)
    s.set_material(w.eps, w.mu)
    s.bind_torch_workspace()
    rng = np.random.default_rng(93)
    K = w.nt
    # a rough state, so that the jumps and the penalty coupling are large
    s.set_state(rng.standard_normal((K, 3, 20)), rng.standard_normal((K, 3, 20)))
    tab = _fullsize_tables(w.verts, w.tets, w.mu, 3, 1.0)
    say(f"[SIP full size] K={K} p=3 fp64 leap-frog CFL 0.2, alpha0 = 1")

    def w_next():
        _, Hp, _ = s.get_state()
        Sp = s.get_sip_state()
        s.step(1)
        E, Hn, _ = s.get_state()
        Sn = s.get_sip_state()
        Wt, Ws = _fullsize_staggered_energy(tab, w.eps, w.mu, E, Hp, Hn, Sp, Sn)
        return Wt, Ws, Sn

    s.step(20)
    W1, Ws1, _ = w_next()
    s.step(100)
    W2, Ws2, Sn = w_next()
    s.close()
    other = tab[2]
    k, f = np.nonzero(other >= 0)
    o = other[k, f]
    dcopy = np.abs(Sn[k, f] - Sn[o // 4, o % 4]).max() / np.abs(Sn).max()
    say(f"  W {W1:.15e} -> {W2:.15e} ({(W2 - W1) / W1:.1e}), h_s share {Ws1 / W1:.2e}, "
        f"copies differ by {dcopy:.1e}")
    assert Ws1 > 1e-3 * W1  # the surface unknown carries energy
    assert abs(W2 - W1) < 1e-11 * W1
    assert dcopy < 1e-12
