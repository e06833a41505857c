"""Pins of the oracle's SIP surface unknown (oracle/sip.py) [KS Sec. III,
eqs. jmp_var_def, 1st_weak_equation, weak_penalty].

* Face basis: orthonormal on the parameter triangle, psi_00 = sqrt(2) and
  psi_01 = 6 s1 - 2 in closed form, and it spans P_p (every monomial of
  degree <= p is reproduced by its projection).
* Face mass in closed form: (mu_F/alpha_F) sqrt(det g) g^-1 (x) I for the
  edge-tangent components (g_kl = t_k . t_l).
* Hand-computed single-face cases: a constant e on one element only gives
  d_t h_s = (alpha_F/mu_F) n x e on each of its faces (the weak penalty
  equation with a constant jump); a constant tangential h_s = tau on one face
  gives the constant E mode -sqrt(6) |F| (tau x n)/(eps J) on both sides.
* Skewness: d/dt of W = 1/2 (eps e, e) + 1/2 (mu h, h) + 1/2 (h_s, M_s h_s)
  vanishes for random states (PEC and interior faces, uneven materials): the
  printed block system [0 C C_F; -C^T 0 0; -C_F^T 0 0]. A wrong jump sign,
  a dropped side, a dropped PEC face or the mirror-ghost jump 2 n x e on PEC
  faces leaves a nonzero rate (each is a one-line check of the rate's face
  sum). A one-sided jump on interior faces keeps skewness but fails the
  consistency pin below.
* Consistency: a global polynomial field of degree <= p has no jumps, so
  d_t h_s = 0 on every interior face.
* Leap-frog with h_s beside h conserves the staggered energy to round-off.
* Purpose: on the unit PEC cube the central scheme has spurious
  eigenfrequencies; with the surface unknown the low spectrum is exactly the
  cavity's.
"""
import numpy as np
import pytest

import workloads as W
from oracle import OracleDG, tri_quadrature
from oracle.sip import SipDG, face_basis, face_modes


def _mesh(seed, n=2):
    verts, tets = W.kuhn_cube_mesh(n, 0.0, 1.0)
    rng = np.random.default_rng(seed)
    verts = W.jitter_interior(verts, 0.0, 1.0, 1.0 / n, 0.1, rng)
    K = len(tets)
    return verts, tets, rng.uniform(1, 4, K), rng.uniform(1, 2, K), rng


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_face_basis_orthonormal_and_complete(p):
    s, w = tri_quadrature(p + 3)
    psi = face_basis(p, s)
    assert psi.shape[1] == (p + 1) * (p + 2) // 2 == len(face_modes(p))
    G = np.einsum("q,qa,qb->ab", w, psi, psi)
    assert np.abs(G - np.eye(psi.shape[1])).max() < 1e-13
    assert np.allclose(psi[:, 0], np.sqrt(2.0))
    if p >= 1:
        assert np.allclose(psi[:, 1], 6.0 * s[:, 0] - 2.0)  # (i, j) = (0, 1)
    # monomials s1^a s2^b, a + b <= p, lie in the span: projection is exact
    mon = np.stack([s[:, 0] ** a * s[:, 1] ** b for a in range(p + 1) for b in range(p + 1 - a)], axis=1)
    proj = psi @ np.einsum("q,qa,qm->am", w, psi, mon)
    assert np.abs(proj - mon).max() < 1e-12


def test_face_mass_closed_form():
    verts, tets, eps, mu, _ = _mesh(3)
    O = OracleDG(verts, tets, 2, eps=eps, mu=mu)
    S = SipDG(O, 0.7)
    NF = S.NF
    for F in (0, 5, S.nfaces - 1):
        t = S.tang[F]
        g = t @ t.T
        M = (S.muF[F] / S.alpha[F]) * np.sqrt(np.linalg.det(g)) * np.kron(np.linalg.inv(g), np.eye(NF))
        assert np.abs(S.mass[F] - M).max() < 1e-12 * np.abs(M).max()


def test_constant_jump_and_constant_surface_field():
    verts, tets, eps, mu, rng = _mesh(5)
    O = OracleDG(verts, tets, 2, eps=eps, mu=mu)
    S = SipDG(O, 1.3)
    K, N = O.K, O.N
    k = 7
    c = np.array([0.3, -1.1, 0.6])
    cE = np.zeros((K, 3, N))
    cE[k, :, 0] = c / np.sqrt(6.0)  # phi_0 = sqrt(6) on the reference tet
    cH = np.zeros((K, 3, N))
    _, _, dS, _, _ = S.rhs(cE, cH, np.zeros((S.nfaces, 2, S.NF)))
    for f in range(4):
        F = S.fid[k, f]
        val = np.einsum("km,kqmi->qi", dS[F], S.vec[F])
        want = (S.alpha[F] / S.muF[F]) * np.cross(O.normal[k, f], c)
        assert np.abs(val - want[None]).max() < 1e-12 * np.abs(want).max()
    # faces not touching element k get nothing
    others = np.setdiff1d(np.arange(S.nfaces), S.fid[k])
    assert np.abs(dS[others]).max() == 0.0
    # a constant tangential h_s = tau on one interior face
    F = next(F for F, (_, _, o) in enumerate(S.sides) if o >= 0)
    (k1, f1, o) = S.sides[F]
    n = O.normal[k1, f1]
    tau = np.cross(n, [0.2, 0.9, -0.4])  # tangential
    Sv = np.zeros((S.nfaces, 2, S.NF))
    Sv[F, :, 0] = S.tang[F] @ tau / np.sqrt(2.0)  # components t_k . tau, psi_00 = sqrt(2)
    dE, _, _, _, _ = S.rhs(np.zeros((K, 3, N)), cH, Sv)
    area = 0.5 * np.linalg.norm(np.cross(S.tang[F][0], S.tang[F][1]))
    dE0, _, _, _ = O.rhs(np.zeros((K, 3, N)), cH)
    for (kk, ff) in ((k1, f1), (o // 4, o % 4)):
        want = -np.sqrt(6.0) * area * np.cross(tau, O.normal[kk, ff]) / (O.eps[kk] * O.J[kk])
        assert np.abs(dE[kk, :, 0] - dE0[kk, :, 0] - want).max() < 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("p", [1, 2])
def test_sip_system_is_skew(p):
    verts, tets, eps, mu, rng = _mesh(7 + p)
    O = OracleDG(verts, tets, p, eps=eps, mu=mu)
    S = SipDG(O, 2.0)
    K, N = O.K, O.N
    cE, cH = rng.standard_normal((K, 3, N)), rng.standard_normal((K, 3, N))
    Sv = rng.standard_normal((S.nfaces, 2, S.NF))
    dE, dH, dS, _, _ = S.rhs(cE, cH, Sv)
    J = O.J[:, None, None]
    a = np.sum(J * eps[:, None, None] * cE * dE)
    b = np.sum(J * mu[:, None, None] * cH * dH)
    c = sum(float(Sv[F].ravel() @ S.mass[F] @ dS[F].ravel()) for F in range(S.nfaces))
    scale = abs(a) + abs(b) + abs(c)
    assert abs(c) > 1e-2 * scale  # the penalty coupling is exercised
    assert abs(a + b + c) < 1e-13 * scale


def test_no_jump_no_penalty_for_global_polynomials():
    verts, tets, eps, mu, rng = _mesh(11)
    O = OracleDG(verts, tets, 3, eps=eps, mu=mu)
    S = SipDG(O, 1.0)

    def fe(x):
        return np.stack([x[..., 1] ** 2 * x[..., 2], x[..., 0] - x[..., 2] ** 3, x[..., 0] * x[..., 1] * x[..., 2]],
                        axis=-1)

    cE = O.project(fe)
    _, _, dS, _, _ = S.rhs(cE, np.zeros_like(cE), np.zeros((S.nfaces, 2, S.NF)))
    inner = np.array([o >= 0 for (_, _, o) in S.sides])
    assert np.abs(dS[inner]).max() < 1e-11
    assert np.abs(dS[~inner]).max() > 1e-2  # PEC faces see n x e


def test_leapfrog_with_sip_conserves_staggered_energy():
    verts, tets, eps, mu, rng = _mesh(13)
    O = OracleDG(verts, tets, 2, eps=eps, mu=mu)
    S = SipDG(O, 1.0)
    K, N = O.K, O.N
    dt = 0.2 * W.cfl_dt(verts, tets, eps, mu, 2, 0.2)
    cE, cH = rng.standard_normal((K, 3, N)), rng.standard_normal((K, 3, N))
    Sv = rng.standard_normal((S.nfaces, 2, S.NF))
    Ws = []
    for n in range(3):
        e1, h1, s1, _, _, _ = S.leapfrog_run(cE, cH, Sv, dt=dt, nsteps=1)
        Ws.append(S.staggered_energy(e1, cH, h1, Sv, s1))
        cE, cH, Sv = e1, h1, s1
        if n == 0:
            cE, cH, Sv, _, _, _ = S.leapfrog_run(cE, cH, Sv, dt=dt, nsteps=30)
    assert abs(Ws[1] - Ws[0]) < 1e-12 * Ws[0] and abs(Ws[2] - Ws[0]) < 1e-12 * Ws[0]


def test_sip_clears_spurious_modes_of_the_cavity():
    """The purpose of the SIP unknown [KS Sec. III]: the central scheme's
    spectrum on the unit PEC cube (6 Kuhn tets, p=3) has eigenfrequencies
    that belong to no cavity mode (below the lowest one, pi sqrt 2); with the
    surface unknown (alpha0 = 1) every eigenfrequency below 6.5 lies within 3%
    of a cavity mode pi sqrt(l^2+m^2+n^2) with its multiplicity (three near
    pi sqrt 2, two near pi sqrt 3), and the spectrum stays on the imaginary
    axis (skew system)."""
    verts, tets = W.kuhn_cube_mesh(1, 0.0, 1.0)
    O = OracleDG(verts, tets, 3)
    S = SipDG(O, 1.0)
    K, N = O.K, O.N
    ne, ns = K * 3 * N, S.nfaces * 2 * S.NF

    def freqs(with_sip):
        n = 2 * ne + (ns if with_sip else 0)
        A = np.zeros((n, n))
        for c in range(n):
            v = np.zeros(n)
            v[c] = 1.0
            E, H = v[:ne].reshape(K, 3, N), v[ne:2 * ne].reshape(K, 3, N)
            if with_sip:
                dE, dH, dS, _, _ = S.rhs(E, H, v[2 * ne:].reshape(S.nfaces, 2, S.NF))
                A[:, c] = np.concatenate([dE.ravel(), dH.ravel(), dS.ravel()])
            else:
                dE, dH, _, _ = O.rhs(E, H)
                A[:, c] = np.concatenate([dE.ravel(), dH.ravel()])
        ev = np.linalg.eigvals(A)
        assert np.abs(ev.real).max() < 1e-10 * np.abs(ev.imag).max()
        return np.sort(ev.imag[ev.imag > 1e-8])

    lowest = np.pi * np.sqrt(2.0)
    plain = freqs(False)
    assert np.sum(plain < 0.97 * lowest) >= 2  # spurious: below every cavity mode
    w = freqs(True)
    w = w[w < 6.5]
    cavity = np.array([lowest] * 3 + [np.pi * np.sqrt(3.0)] * 2)
    assert len(w) == len(cavity)
    assert np.all(np.abs(w / cavity - 1.0) < 0.03)


def test_sip_with_mixed_orders():
    """The paper's pairing (e at order p+1, h and h_s at order p): the block
    system stays skew, global polynomials of e's degree have no jumps, and
    leap-frog conserves the staggered energy."""
    verts, tets, eps, mu, rng = _mesh(17)
    O = OracleDG(verts, tets, 3, eps=eps, mu=mu, ph=2)
    S = SipDG(O, 1.5)
    assert S.NF == 6  # h_s in P_2 of each face
    K = O.K
    cE, cH = rng.standard_normal((K, 3, O.N)), rng.standard_normal((K, 3, O.NH))
    Sv = rng.standard_normal((S.nfaces, 2, S.NF))
    dE, dH, dS, _, _ = S.rhs(cE, cH, Sv)
    J = O.J[:, None, None]
    a = np.sum(J * eps[:, None, None] * cE * dE)
    b = np.sum(J * mu[:, None, None] * cH * dH)
    c = sum(float(Sv[F].ravel() @ S.mass[F] @ dS[F].ravel()) for F in range(S.nfaces))
    scale = abs(a) + abs(b) + abs(c)
    assert abs(c) > 1e-2 * scale and abs(a + b + c) < 1e-13 * scale

    def fe(x):
        return np.stack([x[..., 1] ** 2 * x[..., 2], x[..., 0] - x[..., 2] ** 3, x[..., 0] * x[..., 1] * x[..., 2]],
                        axis=-1)

    _, _, dS0, _, _ = S.rhs(O.project(fe), np.zeros((K, 3, O.NH)), np.zeros_like(Sv))
    inner = np.array([o >= 0 for (_, _, o) in S.sides])
    assert np.abs(dS0[inner]).max() < 1e-11
    dt = 0.2 * W.cfl_dt(verts, tets, eps, mu, 3, 0.2)
    e1, h1, s1, _, _, _ = S.leapfrog_run(cE, cH, Sv, dt=dt, nsteps=1)
    W1 = S.staggered_energy(e1, cH, h1, Sv, s1)
    e2, h2, s2, _, _, _ = S.leapfrog_run(e1, h1, s1, dt=dt, nsteps=20)
    e3, h3, s3, _, _, _ = S.leapfrog_run(e2, h2, s2, dt=dt, nsteps=1)
    W2 = S.staggered_energy(e3, h2, h3, s2, s3)
    assert abs(W2 - W1) < 1e-12 * W1
