"""FP64 CPU oracle for the matrix-free DG Maxwell operator (test infrastructure).

This package is TEST INFRASTRUCTURE ONLY. It may be imported solely by
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py``. The product path (``paper_2002_08733_amd``) never imports it,
and it never imports the product path: the two share no code. The only shared
module is ``workloads`` (seeded meshes, random numbers and closed-form
physical fields, no DG arithmetic).

The oracle computes the semi-discrete DG system of the paper (Sec. III,
eqs. uwc and cwc; Sec. IV, eqs. p_variable / q_variable) in *physical
Cartesian* components with physical quadrature:

* scalar orthonormal Dubiner basis (Sec. II, eq. dubiner_functions in its
  corrected form, see ``basis.py``) pulled back affinely to each element, so
  the Cartesian mass matrix is ``J_T eps_T I``;
* curls by the chain rule at volume quadrature points;
* face integrals at physical face quadrature points with geometric outward
  normals; neighbour values obtained by inverting the neighbour's affine map
  at those points (no reference face matrices, no orientation bookkeeping);
* classic RK4 in time.

Nothing here uses a reference curl matrix, reference trace matrices or a
covariant coefficient frame except in the explicit conversion helpers
(``to_cartesian`` / ``to_covariant``) used to compare with the GPU library.

Parity pins: see ``tests/test_oracle_*.py``. Every function of this package
is pinned by at least one test against mathematics fixed independently of the
oracle (closed forms, textbook identities, brute force, library routines).
"""
from .basis import Dubiner, jacobi, tet_quadrature, tri_quadrature, modes
from .dg import OracleDG, pml_tensors

__all__ = ["Dubiner", "jacobi", "tet_quadrature", "tri_quadrature", "modes",
           "OracleDG", "pml_tensors"]
