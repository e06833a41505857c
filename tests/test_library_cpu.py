"""CPU tests of libmdg's host side: the C ABI loads and exports every symbol
that include/mdg.h declares, mesh topology and error paths, projection points,
and the build-time reference operators pinned against brute-force assembly
with the oracle's basis. No device call is made here."""
import os
import re

import numpy as np
import pytest
from scipy.special import eval_jacobi

import workloads as W
from oracle.basis import Dubiner, tet_quadrature, tri_quadrature

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mdg.h")
GEN_TXT = os.path.join(ROOT, "paper_2002_08733_amd", "csrc", "refops_gen.txt")


def _ensure_built():
    from paper_2002_08733_amd import mdg
    if not os.path.exists(mdg.LIB_PATH) or not os.path.exists(GEN_TXT):
        from paper_2002_08733_amd import build
        build.build()


@pytest.fixture(scope="module")
def lib():
    _ensure_built()
    from paper_2002_08733_amd import mdg
    return mdg


def test_exports_every_declared_symbol(lib):
    names = set(re.findall(r"\b(mdg_[a-z_]+)\s*\(", open(HEADER).read()))
    assert len(names) >= 17
    L = lib.load_library()
    for n in sorted(names):
        assert hasattr(L, n), n
    assert set(lib.SIGNATURES) == names


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_face_counts_on_kuhn_mesh(lib, n):
    v, t = W.kuhn_cube_mesh(n, 0.0, 1.0)
    s = lib.Solver(2)
    s.set_mesh(v, t)
    q = s.query()
    assert q["n_elements"] == 6 * n ** 3
    assert 4 * q["n_elements"] == 2 * q["n_faces_interior"] + q["n_faces_boundary"]
    assert q["n_faces_boundary"] == 12 * n * n


def test_vertex_order_inside_tets_is_irrelevant(lib):
    v, t = W.kuhn_cube_mesh(3, 0.0, 1.0)
    rng = np.random.default_rng(0)
    t2 = np.array([row[rng.permutation(4)] for row in t])
    a, b = lib.Solver(2), lib.Solver(2)
    a.set_mesh(v, t)
    b.set_mesh(v, t2)
    qa, qb = a.query(), b.query()
    for k in ("n_faces_interior", "n_faces_boundary", "n_halo", "n_tiles"):
        assert qa[k] == qb[k]


def test_error_paths(lib):
    v, t = W.kuhn_cube_mesh(1, 0.0, 1.0)
    s = lib.Solver(2)
    with pytest.raises(lib.MdgError) as e:
        s.set_material(np.ones(6), np.ones(6))  # before a mesh
    assert e.value.status == lib.MDG_E_STATE
    bad = t.copy()
    bad[0, 1] = bad[0, 0]
    with pytest.raises(lib.MdgError) as e:
        s.set_mesh(v, bad)
    assert e.value.status == lib.MDG_E_MESH
    flat = v.copy()
    flat[:, 2] = 0.0  # every tet collapses
    with pytest.raises(lib.MdgError) as e:
        s.set_mesh(flat, t)
    assert e.value.status == lib.MDG_E_MESH
    nan = v.copy()
    nan[3, 0] = np.nan
    with pytest.raises(lib.MdgError) as e:
        s.set_mesh(nan, t)
    assert e.value.status == lib.MDG_E_MESH
    oob = t.copy()
    oob[2, 3] = 99
    with pytest.raises(lib.MdgError) as e:
        s.set_mesh(v, oob)
    assert e.value.status == lib.MDG_E_ARG
    # three tets on one face: non-manifold
    vv = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [0, 0, -1], [1, 1, 1.0]])
    tt = np.array([[0, 1, 2, 3], [0, 1, 2, 4], [0, 1, 2, 5]])
    with pytest.raises(lib.MdgError) as e:
        s.set_mesh(vv, tt)
    assert e.value.status == lib.MDG_E_MESH
    s.set_mesh(v, t)
    with pytest.raises(lib.MdgError) as e:
        s.set_material(-np.ones(6), None)
    assert e.value.status == lib.MDG_E_ARG
    with pytest.raises(lib.MdgError) as e:
        s.step(1)
    assert e.value.status == lib.MDG_E_STATE
    # objective and adjoint need a bound workspace too (no device call is made)
    with pytest.raises(lib.MdgError) as e:
        s.probe_energy(3, [0, 1])
    assert e.value.status == lib.MDG_E_STATE
    with pytest.raises(lib.MdgError) as e:
        s.adjoint_probe_energy(3, 1, [0])
    assert e.value.status == lib.MDG_E_STATE
    with pytest.raises(lib.MdgError) as e:
        s.set_dipoles(np.array([[5.0, 5.0, 5.0]]), np.array([[0, 0, 1.0]]), np.array([[2.0, 1.0, 0.4]]))
    assert e.value.status == lib.MDG_E_ARG
    with pytest.raises(lib.MdgError) as e:
        lib.Solver(9)
    assert e.value.status == lib.MDG_E_UNSUPPORTED


def test_projection_points_inside_elements(lib):
    v, t = W.kuhn_cube_mesh(2, -1.0, 1.0)
    rng = np.random.default_rng(1)
    v = W.jitter_interior(v, -1.0, 1.0, 1.0, 0.1, rng)
    s = lib.Solver(3)
    s.set_mesh(v, t)
    x = s.projection_points(4)
    assert x.shape == (len(t), 64, 3)
    X = v[np.sort(t, axis=1)]
    A = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    r = np.einsum("kij,kqj->kqi", np.linalg.inv(A), x - X[:, None, 0])
    assert r.min() > 0 and (1 - r.sum(axis=2)).min() > 0


def test_cfl_step_matches_rule(lib):
    v, t = W.kuhn_cube_mesh(4, 0.0, 1.0)
    s = lib.Solver(2, cfl=0.3)
    s.set_mesh(v, t)
    ones = np.ones(len(t))
    assert abs(s.query()["dt"] - W.cfl_dt(v, t, ones, ones, 2, 0.3)) < 1e-15


def _read_gen():
    D, T = {}, {}
    for line in open(GEN_TXT):
        k, p, a, b, c, val = line.split()
        p, a, b, c = int(p), int(a), int(b), int(c)
        (D if k == "D" else T).setdefault(p, {})[(a, b, c)] = float(val)
    return D, T


def _psi(i, j, s1, s2):
    # orthonormal face basis of the library, written out independently
    b = np.where(np.abs(1 - s1) > 1e-300, 2 * s2 / np.where(np.abs(1 - s1) > 1e-300, 1 - s1, 1) - 1, -1)
    return (np.sqrt(2 * (2 * i + 1) * (i + j + 1)) * eval_jacobi(i, 0, 0, b) * (1 - s1) ** i
            * eval_jacobi(j, 2 * i + 1, 0, 2 * s1 - 1))


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_generated_reference_operators(lib, p):
    """D_a[l][m] = (d_a phi_l, phi_m) and T_f[m][l] = int psi_m phi_l(F_f(s)) ds
    of the generated header equal brute-force quadrature with the oracle's
    basis; structural zeros are exact zeros."""
    D, T = _read_gen()
    B = Dubiner(p)
    N = B.N
    q, w = tet_quadrature(p + 2)
    Dref = np.einsum("q,qal,qm->alm", w, B.grad(q), B.eval(q))
    Dg = np.zeros((3, N, N))
    for (a, l, m), val in D[p].items():
        Dg[a, l, m] = val
    np.testing.assert_allclose(Dg, Dref, atol=1e-12 * max(1, np.abs(Dref).max()))
    assert np.all((Dg == 0) == (np.abs(Dref) < 1e-10))
    fm = [(i, d - i) for d in range(p + 1) for i in range(d + 1)]
    sq, sw = tri_quadrature(p + 2)
    verts = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]])
    NF = len(fm)
    Tg = np.zeros((4, NF, N))
    for (f, m, l), val in T[p].items():
        Tg[f, m, l] = val
    for f in range(4):
        a, b, c = verts[[v for v in range(4) if v != f]]
        pts = a + sq[:, :1] * (b - a) + sq[:, 1:] * (c - a)
        ph = B.eval(pts)
        ps = np.array([_psi(i, j, sq[:, 0], sq[:, 1]) for (i, j) in fm])
        Tref = np.einsum("q,mq,ql->ml", sw, ps, ph)
        np.testing.assert_allclose(Tg[f], Tref, atol=1e-12 * max(1, np.abs(Tref).max()))
        assert np.all((Tg[f] == 0) == (np.abs(Tref) < 1e-10))


def test_instances_host_side(lib):
    w = W.batched(3, 2, seed=11, nmin=2, nmax=4)
    first = w.info["first"]
    s = lib.Solver(2, "fp32", "upwind", tile=32)
    s.set_mesh(w.verts, w.tets)
    s.set_instances(first)
    pos = np.array([d[0] for d in w.dipoles])
    dr = np.array([d[1] for d in w.dipoles])
    wave = np.array([[2.0, 1.0, 5.0 / (2 * np.pi)]] * len(w.dipoles))
    s.set_dipoles(pos, dr, wave, instance=[d[3] for d in w.dipoles])
    assert s.workspace_size() > 0
    q = s.query()
    assert q["n_instances"] == 3 and q["n_dipoles"] == 3 and q["tile_size"] == 32
    # the instances' elements stay together: no halo face can join two of
    # them, and the face count is the sum of the instances'
    nb = sum(12 * int(n) ** 2 for n in w.info["sizes"])
    assert q["n_faces_boundary"] == nb
    # errors
    with pytest.raises(lib.MdgError) as e:
        s.set_instances(np.array([1, w.nt]))
    assert e.value.status == lib.MDG_E_ARG
    with pytest.raises(lib.MdgError) as e:
        s.set_instances(np.array([0, w.nt - 1]))
    assert e.value.status == lib.MDG_E_ARG
    with pytest.raises(lib.MdgError) as e:
        s.set_instances(np.array([0, 5, 5, w.nt]))
    assert e.value.status == lib.MDG_E_ARG
    with pytest.raises(lib.MdgError) as e:
        s.set_dipoles(pos[:1], dr[:1], wave[:1], instance=[7])
    assert e.value.status == lib.MDG_E_ARG
    # a point of instance 0's region that lies outside instance 2's box cannot be found there
    with pytest.raises(lib.MdgError) as e:
        s.set_dipoles(np.array([[5.0, 5.0, 5.0]]), dr[:1], wave[:1], instance=[2])
    assert e.value.status == lib.MDG_E_ARG
    s.close()


def test_instances_must_not_share_faces(lib):
    v, t = W.kuhn_cube_mesh(2, 0.0, 1.0)
    s = lib.Solver(1)
    s.set_mesh(v, t)
    with pytest.raises(lib.MdgError) as e:
        s.set_instances(np.array([0, 24, 48]))
    assert e.value.status == lib.MDG_E_MESH
    s.close()


def test_tile_option_is_validated(lib):
    with pytest.raises(lib.MdgError) as e:
        lib.Solver(2, tile=48)
    assert e.value.status == lib.MDG_E_ARG


def test_integrator_option_is_validated(lib):
    # leap-frog shares one halo buffer between its halves, which is exact
    # only when a field's derivative reads no trace of that field (central flux)
    with pytest.raises(lib.MdgError) as e:
        lib.Solver(2, flux="upwind", integrator="leapfrog")
    assert e.value.status == lib.MDG_E_UNSUPPORTED
    s = lib.Solver(2, flux="central", integrator="leapfrog", dt=1e-3)
    s.close()
    o = lib.mdg_options(order=2, precision=lib.MDG_FP64, flux=lib.MDG_CENTRAL, integrator=7, dt=1e-3, cfl=0.0,
                        tile=0, mixed=0)
    h = lib._VP()
    assert lib.load_library().mdg_create(lib.ctypes.byref(o), lib.ctypes.byref(h)) == lib.MDG_E_ARG


def test_leapfrog_bytes_per_half_step(lib):
    # a leap-frog half step reads both fields and writes one: 9/(17/4 * 6) of
    # an RK4 stage's state traffic
    verts, tets = W.kuhn_cube_mesh(3)
    q = {}
    for integ in ("rk4", "leapfrog"):
        s = lib.Solver(2, flux="central", integrator=integ, dt=1e-3)
        s.set_mesh(verts, tets)
        s.workspace_size()
        q[integ] = s.query()["bytes_per_stage"]
        s.close()
    K, N, rs = len(tets), 10, 8
    geo = 9 * rs + 16
    assert q["rk4"] == pytest.approx(K * (17 / 4 * 6 * N * rs + geo))
    assert q["leapfrog"] == pytest.approx(K * (9 * N * rs + geo))


def test_mixed_order_option(lib):
    with pytest.raises(lib.MdgError) as e:
        lib.Solver(4, mixed=True)  # e would need order 5
    assert e.value.status == lib.MDG_E_UNSUPPORTED
    o = lib.mdg_options(order=2, precision=lib.MDG_FP64, flux=lib.MDG_CENTRAL, integrator=0, dt=1e-3, cfl=0.0,
                        tile=0, mixed=2)
    h = lib._VP()
    assert lib.load_library().mdg_create(lib.ctypes.byref(o), lib.ctypes.byref(h)) == lib.MDG_E_ARG
    s = lib.Solver(2, mixed=True, dt=1e-3)
    q = s.query()
    assert (q["order"], q["nmodes"], q["order_h"], q["nmodes_h"]) == (3, 20, 2, 10)
    # algorithmic bytes count the modes of h at its own order
    verts, tets = W.kuhn_cube_mesh(2)
    s.set_mesh(verts, tets)
    s.workspace_size()
    geo = 9 * 8 + 16
    assert s.query()["bytes_per_stage"] == pytest.approx(len(tets) * (17 / 4 * 3 * (20 + 10) * 8 + geo))
    s.close()
    s = lib.Solver(2, dt=1e-3)
    q = s.query()
    assert (q["order"], q["nmodes"], q["order_h"], q["nmodes_h"]) == (2, 10, 2, 10)
    s.close()


def test_sip_option_and_host_side_errors(lib):
    verts, tets = W.kuhn_cube_mesh(2)
    # the SIP unknown comes with the central flux
    with pytest.raises(lib.MdgError) as e:
        lib.Solver(2, dt=1e-3, sip_alpha=1.0, flux="upwind")
    assert e.value.status == lib.MDG_E_UNSUPPORTED
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(lib.MdgError) as e:
            lib.Solver(2, dt=1e-3, sip_alpha=bad)
        assert e.value.status == lib.MDG_E_ARG
    # state calls on a solver without it; instances; operator-only calls
    s = lib.Solver(2, dt=1e-3)
    s.set_mesh(verts, tets)
    z = np.zeros((len(tets), 3, 10))
    for call in (s.get_sip_state, lambda: s.rhs_sip(z, z)):
        with pytest.raises(lib.MdgError) as e:
            call()
        assert e.value.status == lib.MDG_E_UNSUPPORTED
    s.close()
    s = lib.Solver(2, dt=1e-3, sip_alpha=1.0)
    s.set_mesh(verts, tets)
    K, N = len(tets), 10
    z = np.zeros((K, 3, N))
    with pytest.raises(lib.MdgError) as e:
        s.rhs(z, z)  # the SIP unknown needs mdg_rhs_sip
    assert e.value.status == lib.MDG_E_UNSUPPORTED
    # algorithmic bytes: 8 NF surface values per element streamed like the
    # state, plus the four face rows of the geometry record
    s.workspace_size()
    NF, rs = 6, 8
    geo = 9 * rs + 16
    want = K * (17 / 4 * 6 * N * rs + geo + 17 / 4 * 8 * NF * rs + 4 * rs)
    assert s.query()["bytes_per_stage"] == pytest.approx(want)
    s.close()
    # mixed orders (e order 3, h order 2): h_s has the face modes of order 2
    s = lib.Solver(2, dt=1e-3, sip_alpha=1.0, mixed=True, integrator="leapfrog")
    s.set_mesh(verts, tets)
    s.workspace_size()
    assert s.nfacemodes == 6
    want = K * (4.5 * (20 + 10) * rs + geo + 12 * 6 * rs + 4 * rs)
    assert s.query()["bytes_per_stage"] == pytest.approx(want)
    s.close()


def test_empty_and_oversized_meshes(lib):
    """Edge cases of the decomposition: an empty mesh is refused, and a mesh
    whose state array passes 4 GiB is accepted (the stage kernel addresses
    every element array through per-tile windows): FP64 at order 4 holds
    6 x 35 x 8 bytes per element, so 2,633,856 tets (76^3 cubes) need 4.4 GB
    for one state array."""
    s = lib.Solver(2, dt=1e-3)
    v, t = W.kuhn_cube_mesh(1, 0.0, 1.0)
    with pytest.raises(lib.MdgError) as e:
        s.set_mesh(v, t[:0])
    assert e.value.status == lib.MDG_E_ARG
    s.close()
    v, t = W.kuhn_cube_mesh(76, 0.0, 1.0)
    s = lib.Solver(4, "fp64", dt=1e-3)
    s.set_mesh(v, t)
    assert s.workspace_size() > 4 * (4 << 30)
    s.close()
    # the same mesh in FP32 at order 3 (2.1 GB per state array) is accepted
    s = lib.Solver(3, "fp32", dt=1e-3)
    s.set_mesh(v, t)
    assert s.workspace_size() > 4 * 6 * 20 * 4 * len(t)
    s.close()


def test_monitor_option_is_checked(lib):
    """mdg_options.monitor: 0 or >= 2 (RK4 is strongly stable over two steps)."""
    for bad in (1, -3):
        with pytest.raises(lib.MdgError) as e:
            lib.Solver(2, monitor=bad)
        assert e.value.status == lib.MDG_E_ARG
    lib.Solver(2, monitor=2).close()


def test_mfma_option_is_checked(lib):
    """mdg_options.mfma: FP32, RK4, order <= 3 and 64-element tiles only."""
    lib.Solver(3, "fp32", mfma=True).close()
    for kw in (dict(precision="fp64"), dict(precision="fp32", integrator="leapfrog"),
               dict(precision="fp32", tile=32)):
        with pytest.raises(lib.MdgError) as e:
            lib.Solver(3, mfma=True, **kw)
        assert e.value.status == lib.MDG_E_UNSUPPORTED
    with pytest.raises(lib.MdgError) as e:
        lib.Solver(4, "fp32", mfma=True)
    assert e.value.status == lib.MDG_E_UNSUPPORTED


def _cross_tile_faces(verts, tets, tile_of):
    """Interior faces whose two elements lie in different tiles (counted once
    per side, like the library's halo slots)."""
    f = np.sort(np.stack([tets[:, [1, 2, 3]], tets[:, [0, 2, 3]], tets[:, [0, 1, 3]], tets[:, [0, 1, 2]]], axis=1),
                axis=2).reshape(-1, 3)
    key = (f[:, 0].astype(np.int64) * len(verts) + f[:, 1]) * len(verts) + f[:, 2]
    o = np.argsort(key, kind="stable")
    same = np.nonzero(key[o][1:] == key[o][:-1])[0]
    a, b = o[same] // 4, o[same + 1] // 4
    return 2 * int(np.count_nonzero(tile_of[a] != tile_of[b]))


def test_tile_order_cuts_compact_tiles(lib):
    """Tiles are runs of the element order (setup.cpp::finalize): on the
    jittered cube the bisection order must give fewer cross-tile faces than
    cutting the same mesh along a plain lexicographic order of centroids
    would, and on the open-domain mesh, whose PML shell is hollow, the order
    must keep 64-element FP32 tiles (a bisection leaf that spans the hole has
    only halo faces, and the largest halo block sizes every workgroup's LDS)."""
    w = W.jittered(16, 3, seed=2, flux="upwind")
    s = lib.Solver(3, "fp32", "upwind", dt=1e-4)
    s.set_mesh(w.verts, w.tets)
    q = s.query()
    s.close()
    assert q["tile_size"] == 64
    cen = w.verts[w.tets].mean(axis=1)
    lex = np.lexsort((cen[:, 0], cen[:, 1], cen[:, 2]))
    tile_of = np.empty(len(w.tets), np.int64)
    tile_of[lex] = np.arange(len(w.tets)) // 64
    assert q["n_halo"] < 0.8 * _cross_tile_faces(w.verts, w.tets, tile_of)
    wp = W.open_pml(48, 3)  # the open-domain configuration (663,552 tets; 3 s on the host)
    s = lib.Solver(3, "fp32", "upwind", dt=1e-4)
    s.set_mesh(wp.verts, wp.tets)
    s.set_pml(wp.omega)
    qp = s.query()
    s.close()
    assert qp["tile_size"] == 64 and qp["n_pml"] > 0
