"""Shared helpers of the GPU parity tests: build a library solver and an oracle
on the same seeded inputs and compare them in the oracle's Cartesian frame."""
import sys

import numpy as np

import workloads as W
from oracle import OracleDG


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def unit_jittered(n, seed, lo=0.0, hi=1.0, mu_var=True):
    verts, tets = W.kuhn_cube_mesh(n, lo, hi)
    rng = np.random.default_rng(seed)
    verts = W.jitter_interior(verts, lo, hi, (hi - lo) / n, 0.1, rng)
    eps = rng.uniform(1.0, 4.0, len(tets))
    mu = rng.uniform(1.0, 2.0, len(tets)) if mu_var else np.ones(len(tets))
    return verts, tets, eps, mu


def dipole_args(dipoles):
    pos = np.array([d[0] for d in dipoles], dtype=np.float64)
    dr = np.array([d[1] for d in dipoles], dtype=np.float64)
    wave = np.array([[d[2][0], d[2][1], 5.0 / (2 * np.pi * d[2][1])] for d in dipoles])
    return pos, dr, wave


def oracle_dipoles(dipoles):
    return [(d[0], d[1], (lambda t, f0=d[2][0], bw=d[2][1]: W.dipole_waveform(t, f0, bw))) for d in dipoles]


def make_pair(verts, tets, p, flux, precision="fp64", eps=None, mu=None, omega=None, dipoles=(), dt=1e-3):
    from paper_2002_08733_amd import Solver
    s = Solver(p, precision, flux, dt=dt)
    s.set_mesh(verts, tets)
    s.set_material(eps, mu)
    if omega is not None:
        s.set_pml(omega)
    if dipoles:
        s.set_dipoles(*dipole_args(dipoles))
    s.bind_torch_workspace()
    O = OracleDG(verts, tets, p, eps=eps, mu=mu, flux=flux, omega=omega,
                 dipoles=oracle_dipoles(dipoles))
    return s, O


def rel_energy_err(O, aE, aH, bE, bH, aP=None, aQ=None, bP=None, bQ=None, elementwise=True):
    """Relative error of a against b in the energy norm (Cartesian
    coefficients): sqrt(sum J (eps |dE|^2 + mu |dH|^2 [+ |dP|^2/eps + |dQ|^2/mu]))
    over the same of b. With elementwise (default) the larger of that and the
    per-element maximum, max_T ||a - b||_T / max_T ||b||_T, so that one bad
    element cannot hide in the global sum."""
    J, e, m = O.J[:, None, None], O.eps[:, None, None], O.mu[:, None, None]

    def nrm2(E, H, P, Q):  # per element; E, P and H, Q may differ in modes (mixed orders)
        v = np.sum(J * e * E * E, axis=(1, 2)) + np.sum(J * m * H * H, axis=(1, 2))
        if P is not None:
            v += np.sum(J * P * P / e, axis=(1, 2)) + np.sum(J * Q * Q / m, axis=(1, 2))
        return v

    dP = None if aP is None else aP - bP
    dQ = None if aQ is None else aQ - bQ
    d2, b2 = nrm2(aE - bE, aH - bH, dP, dQ), nrm2(bE, bH, bP, bQ)
    err = np.sqrt(d2.sum() / b2.sum())
    if elementwise:
        err = max(err, np.sqrt(d2.max() / b2.max()))
    return err


def element_energy(verts, tets, eps, mu, E, H, P=None, Q=None, chunk=1 << 18):
    """Per-element energy 1/2 (eps u.M u + mu f.M f [+ p.M p / eps + q.M q / mu])
    of covariant coefficients [nt][3][N] in the canonical element frame
    (vertices in ascending id order, A = [v1-v0, v2-v0, v3-v0]), with
    M = |det A| A^-1 A^-T: the L2 norm of the Cartesian field A^-T u. Written
    from the mesh alone, independent of the library's energy reduction."""
    out = np.empty(len(tets))
    for s in range(0, len(tets), chunk):
        sl = slice(s, s + chunk)
        X = verts[np.sort(tets[sl], axis=1)]
        A = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
        Ai = np.linalg.inv(A)
        M = np.abs(np.linalg.det(A))[:, None, None] * (Ai @ np.transpose(Ai, (0, 2, 1)))

        def q(U):
            return np.einsum("kim,kij,kjm->k", U[sl], M, U[sl])

        w = eps[sl] * q(E) + mu[sl] * q(H)
        if P is not None:
            w += q(P) / eps[sl] + q(Q) / mu[sl]
        out[sl] = 0.5 * w
    return out


def rel_state_err(verts, tets, eps, mu, a, b):
    """Relative energy-norm difference of covariant states a, b (tuples E, H
    [, P, Q]): the larger of sqrt(sum_T W_T(a - b) / sum_T W_T(b)) and the
    per-element sqrt(max_T W_T(a - b) / max_T W_T(b)), so that one bad element
    cannot hide in the global sum."""
    d = element_energy(verts, tets, eps, mu, *[x - y for x, y in zip(a, b)])
    r = element_energy(verts, tets, eps, mu, *b)
    return float(max(np.sqrt(d.sum() / r.sum()), np.sqrt(d.max() / r.max())))


def element_bilinear(verts, tets, eps, mu, a, b, chunk=1 << 18):
    """Per-element eps a_E.M b_E + mu a_H.M b_H of covariant coefficient
    pairs a = (E, H), b = (E, H) (canonical frame, M as in element_energy)."""
    out = np.empty(len(tets))
    for s in range(0, len(tets), chunk):
        sl = slice(s, s + chunk)
        X = verts[np.sort(tets[sl], axis=1)]
        A = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
        Ai = np.linalg.inv(A)
        M = np.abs(np.linalg.det(A))[:, None, None] * (Ai @ np.transpose(Ai, (0, 2, 1)))
        out[sl] = (eps[sl] * np.einsum("kim,kij,kjm->k", a[0][sl], M, b[0][sl])
                   + mu[sl] * np.einsum("kim,kij,kjm->k", a[1][sl], M, b[1][sl]))
    return out
