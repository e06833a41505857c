"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the DG method: it only builds meshes,
draws random numbers and defines closed-form physical fields that both the
oracle and the GPU library then project / evaluate with their own code.

Workloads (structured stand-ins for the paper's Netgen meshes, Sec. V):

* ``cavity``   : PEC unit cube [0,1]^3, n^3 Kuhn cubes x 6 tets, vacuum.
* ``jittered`` : cube [-1,1]^3, n^3 Kuhn cubes, interior vertices jittered by
                 U(-0.1h, 0.1h) per coordinate, eps ~ U[1,4] per element.
* ``open_pml`` : inner box [-1,1]^3 plus a PML shell of ``nl`` elements,
                 per-element per-axis damping sampled at the centroid.

All random draws use ``numpy.random.default_rng(seed)`` in the fixed order
(vertex jitter, then permittivity, then anything else).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np


# ---------------------------------------------------------------------------
# meshes
# ---------------------------------------------------------------------------

def kuhn_cube_mesh(n: int, lo: float = 0.0, hi: float = 1.0):
    """Structured tetrahedral mesh of the cube [lo,hi]^3 with n^3 sub-cubes.

    Every sub-cube is split into the 6 Kuhn (Freudenthal) tetrahedra: one per
    permutation of the axes, each a monotone lattice path from the cube's low
    corner to its high corner. The triangulation is conforming.

    Returns ``(verts[nv,3] float64, tets[nt,4] int64)``. Vertex id of lattice
    point (i,j,k) is ``i + (n+1)*(j + (n+1)*k)``; tets are listed cube by cube
    (x fastest), six per cube.
    """
    m = n + 1
    g = np.linspace(lo, hi, m)
    lat = np.arange(m)
    # vertex (i,j,k) -> id i + m*(j + m*k): x fastest
    K, J, I = np.meshgrid(lat, lat, lat, indexing="ij")
    verts = np.stack([g[I.ravel()], g[J.ravel()], g[K.ravel()]], axis=1)
    c = np.arange(n)
    CK, CJ, CI = np.meshgrid(c, c, c, indexing="ij")
    low = np.stack([CI.ravel(), CJ.ravel(), CK.ravel()], axis=1)  # cube low corners, x fastest
    tets = np.empty((low.shape[0], 6, 4), dtype=np.int64)
    for t, perm in enumerate(itertools.permutations(range(3))):
        cur = low.copy()
        tets[:, t, 0] = cur[:, 0] + m * (cur[:, 1] + m * cur[:, 2])
        for s, ax in enumerate(perm):
            cur[:, ax] += 1
            tets[:, t, s + 1] = cur[:, 0] + m * (cur[:, 1] + m * cur[:, 2])
    tets = tets.reshape(-1, 4)
    return verts, tets


def boundary_vertex_mask(verts: np.ndarray, lo: float, hi: float, tol: float = 1e-12):
    """True for vertices on the boundary of the box [lo,hi]^3."""
    return np.any((np.abs(verts - lo) < tol) | (np.abs(verts - hi) < tol), axis=1)


def jitter_interior(verts, lo, hi, h, amount, rng):
    """Move every interior vertex by U(-amount*h, amount*h) per coordinate."""
    out = verts.copy()
    inner = ~boundary_vertex_mask(verts, lo, hi)
    d = rng.uniform(-amount * h, amount * h, size=(int(inner.sum()), 3))
    out[inner] += d
    return out


def tet_centroids(verts, tets):
    return verts[tets].mean(axis=1)


def tets_with_vertex(tets, vid):
    """Indices of the tets that have ``vid`` as a vertex (ascending)."""
    return np.nonzero(np.any(tets == vid, axis=1))[0]


# ---------------------------------------------------------------------------
# closed-form physical fields (inputs; each side projects them itself)
# ---------------------------------------------------------------------------

def te101_fields(x, t=0.0):
    """TE101 eigenmode of the PEC unit cube, eps = mu = 1 (textbook closed form).

    e = y_hat sin(pi x) sin(pi z) cos(w t)
    h = (pi/w) sin(w t) (sin(pi x) cos(pi z), 0, -cos(pi x) sin(pi z))
    with w = pi*sqrt(2). ``x`` is [..., 3]; returns (e, h) of the same shape.
    """
    w = np.pi * np.sqrt(2.0)
    X, Z = x[..., 0], x[..., 2]
    e = np.zeros_like(x)
    e[..., 1] = np.sin(np.pi * X) * np.sin(np.pi * Z) * np.cos(w * t)
    h = np.zeros_like(x)
    c = (np.pi / w) * np.sin(w * t)
    h[..., 0] = c * np.sin(np.pi * X) * np.cos(np.pi * Z)
    h[..., 2] = -c * np.cos(np.pi * X) * np.sin(np.pi * Z)
    return e, h


def te101_omega():
    return np.pi * np.sqrt(2.0)


def gaussian_curl_e(x, width=0.2, center=(0.0, 0.0, 0.0)):
    """Divergence-free pulse e0 = curl(z_hat g), g = exp(-|r-c|^2/w^2).

    curl(z_hat g) = (dg/dy, -dg/dx, 0) = g * (-2 y / w^2, 2 x / w^2, 0).
    """
    r = x - np.asarray(center)
    g = np.exp(-np.sum(r * r, axis=-1) / width**2)
    e = np.zeros_like(x)
    e[..., 0] = -2.0 * r[..., 1] / width**2 * g
    e[..., 1] = 2.0 * r[..., 0] / width**2 * g
    return e


def dipole_waveform(t, f0=2.0, bw=1.0):
    """Gaussian-modulated sinusoid g(t) = sin(2 pi f0 (t-t0)) exp(-(t-t0)^2/(2 s^2)).

    s = 1/(2 pi bw), t0 = 5 s.
    """
    s = 1.0 / (2.0 * np.pi * bw)
    t0 = 5.0 * s
    return np.sin(2.0 * np.pi * f0 * (t - t0)) * np.exp(-((t - t0) ** 2) / (2.0 * s * s))


def random_coefficients(nt, nmodes, seed, ncomp=3):
    """Seeded N(0,1) coefficient array [nt, ncomp, nmodes]."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nt, ncomp, nmodes))


def nmodes(p: int) -> int:
    """Number of scalar modes of P_p on a tetrahedron, C(p+3,3)."""
    return (p + 1) * (p + 2) * (p + 3) // 6


# ---------------------------------------------------------------------------
# workload recipes
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    verts: np.ndarray
    tets: np.ndarray
    p: int
    eps: np.ndarray
    mu: np.ndarray
    flux: str  # "central" | "upwind"
    omega: np.ndarray | None = None  # [nt,3] PML damping per element, or None
    dipoles: list = field(default_factory=list)  # (pos[3], dir[3], (f0,bw))
    h: float = 0.0
    box: tuple = (0.0, 1.0)
    steps: int = 0
    cfl: float = 0.3
    info: dict = field(default_factory=dict)

    @property
    def nt(self):
        return self.tets.shape[0]


def cavity(n=4, p=2):
    """PEC unit cube, n^3 Kuhn cubes, vacuum, central flux (TE101 test case)."""
    verts, tets = kuhn_cube_mesh(n, 0.0, 1.0)
    nt = tets.shape[0]
    return Workload(f"cavity_n{n}_p{p}", verts, tets, p, np.ones(nt), np.ones(nt),
                    "central", h=1.0 / n, box=(0.0, 1.0), steps=100)


def jittered(n=32, p=3, seed=2, flux="upwind", amount=0.1):
    """[-1,1]^3, n^3 Kuhn cubes, interior jitter U(-0.1h,0.1h), eps ~ U[1,4]."""
    verts, tets = kuhn_cube_mesh(n, -1.0, 1.0)
    h = 2.0 / n
    rng = np.random.default_rng(seed)
    verts = jitter_interior(verts, -1.0, 1.0, h, amount, rng)
    eps = rng.uniform(1.0, 4.0, size=tets.shape[0])
    mu = np.ones(tets.shape[0])
    return Workload(f"jittered_n{n}_p{p}", verts, tets, p, eps, mu, flux, h=h,
                    box=(-1.0, 1.0), steps=1000)


def batched(n_inst=64, p=3, seed=4, nmin=8, nmax=24, flux="upwind", amount=0.1):
    """Independent instances for one batched solver. Instance i: [-1,1]^3 with
    n_i^3 Kuhn cubes, n_i ~ U{nmin..nmax}, interior jitter U(-0.1h, 0.1h), its
    own eps ~ U[1,4], mu = 1, and a z-directed dipole (f0 = 2, bw = 1) at a
    point ~ U([-0.5,0.5]^3). The meshes are concatenated with offset vertex
    ids; info["first"] holds the element range of every instance and each
    dipole carries its instance index as a fourth entry. rng order per
    instance: size (drawn first for all), jitter, eps, dipole point."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(nmin, nmax + 1, size=n_inst)
    V, T, E, dips, first = [], [], [], [], [0]
    voff = 0
    for i, n in enumerate(sizes):
        n = int(n)
        verts, tets = kuhn_cube_mesh(n, -1.0, 1.0)
        verts = jitter_interior(verts, -1.0, 1.0, 2.0 / n, amount, rng)
        E.append(rng.uniform(1.0, 4.0, size=tets.shape[0]))
        pos = rng.uniform(-0.5, 0.5, size=3)
        dips.append((pos, np.array([0.0, 0.0, 1.0]), (2.0, 1.0), i))
        V.append(verts)
        T.append(tets + voff)
        voff += verts.shape[0]
        first.append(first[-1] + tets.shape[0])
    verts = np.concatenate(V)
    tets = np.concatenate(T)
    eps = np.concatenate(E)
    return Workload(f"batched_{n_inst}x_p{p}", verts, tets, p, eps, np.ones(tets.shape[0]), flux,
                    dipoles=dips, box=(-1.0, 1.0), steps=500,
                    info={"first": np.array(first, dtype=np.int64), "sizes": sizes})


def pml_profile(centroids, inner=1.0, thickness=0.2, sigma_max=20.0, power=3):
    """Per-element, per-axis damping w_a = sigma_max (d_a/L)^power at the centroid,
    d_a = max(0, |x_a| - inner), L = thickness. Zero inside the inner box."""
    d = np.maximum(0.0, np.abs(centroids) - inner)
    return sigma_max * (d / thickness) ** power


def open_pml(n=48, p=3, layers=4, inner=1.0, sigma_max=20.0, flux="upwind"):
    """Inner box [-1,1]^3 + PML shell of ``layers`` elements, vacuum, z-dipole."""
    hcell = inner / (n / 2 - layers)
    outer = inner + layers * hcell
    verts, tets = kuhn_cube_mesh(n, -outer, outer)
    nt = tets.shape[0]
    cen = tet_centroids(verts, tets)
    omega = pml_profile(cen, inner, layers * hcell, sigma_max)
    # dipole at the origin: a mesh vertex, moved to the centroid of the
    # lowest-index tet that has it as a vertex
    origin = int(np.argmin(np.sum(verts**2, axis=1)))
    t0 = int(tets_with_vertex(tets, origin)[0])
    pos = cen[t0]
    dip = [(pos, np.array([0.0, 0.0, 1.0]), (2.0, 1.0))]
    return Workload(f"open_pml_n{n}_p{p}", verts, tets, p, np.ones(nt), np.ones(nt),
                    flux, omega=omega, dipoles=dip, h=hcell, box=(-outer, outer),
                    steps=2000, info={"inner": inner, "layers": layers,
                                      "sigma_max": sigma_max, "dipole_tet": t0})


def containing_tet(verts, tets, x, tol=1e-12):
    """Lowest-index tet whose closure contains the point x (barycentric test)."""
    X = verts[tets]  # [nt,4,3]
    A = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    lam = np.linalg.solve(A, (np.asarray(x, dtype=np.float64)[None, :] - X[:, 0])[:, :, None])[:, :, 0]
    bary = np.concatenate([1.0 - lam.sum(axis=1, keepdims=True), lam], axis=1)
    idx = np.flatnonzero(np.all(bary >= -tol, axis=1))
    if idx.size == 0:
        raise ValueError("point outside the mesh")
    return int(idx[0])


def adjoint_pml(n=24, p=3, layers=3):
    """The adjoint workload: open_pml with n^3 cubes (inner [-1,1]^3 of n-2*layers
    cubes per axis plus a PML ``layers`` cubes thick), central flux, the z-dipole
    at the origin, and 8 probe elements: the lowest-index tet containing each
    point (+-1/2, +-1/2, +-1/2)."""
    w = open_pml(n, p, layers=layers, flux="central")
    probes = [containing_tet(w.verts, w.tets, np.array([sx, sy, sz]))
              for sx in (-0.5, 0.5) for sy in (-0.5, 0.5) for sz in (-0.5, 0.5)]
    w.info["probes"] = np.array(probes, dtype=np.int64)
    w.name = f"adjoint_pml_n{n}_p{p}"
    return w


def cfl_dt(verts, tets, eps, mu, p, cfl):
    """Explicit step from a CFL number: dt = cfl * min_T(2 r_in sqrt(eps mu)) / (p+1)^2,
    r_in = 3|T| / (sum of face areas). Mesh geometry only (no DG arithmetic)."""
    x = verts[tets]
    a, b, c, d = x[:, 0], x[:, 1], x[:, 2], x[:, 3]
    vol = np.abs(np.einsum("ij,ij->i", b - a, np.cross(c - a, d - a))) / 6.0
    def area(p0, p1, p2):
        return 0.5 * np.linalg.norm(np.cross(p1 - p0, p2 - p0), axis=1)
    s = area(b, c, d) + area(a, c, d) + area(a, b, d) + area(a, b, c)
    rin = 3.0 * vol / s
    return float(cfl * np.min(2.0 * rin * np.sqrt(eps * mu)) / (p + 1) ** 2)
