"""Plain FP64 CPU oracle for the wedge/tet nodal DG acoustic solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, tables or
constants with the HIP library; both sides are written independently from
the paper (Chan, Wang, Hewett, Warburton, "Reduced storage nodal
discontinuous Galerkin methods on semi-structured prismatic meshes").

The oracle computes the *plain definition* of the method: the strong-form
DG semi-discretisation of Sec. 2 (eq. ``form``) with every element matrix
(mass, weak derivatives, face integrals) evaluated by quadrature that is
exact for vertically mapped wedges, and the mass matrix inverted densely.
None of the Kronecker/Lemma-1 structure of Sec. 3-4 is used, which is what
lets the tests pin that structure against it.

Modules
-------
basis     1D GLL/Gauss, triangle Warp & Blend nodes, Lagrange bases, quadrature
geometry  wedge vertex map, Jacobians, inverse map by Newton iteration
dg        connectivity, dense element operators, RHS, energy, sources
lsrk      five-stage fourth-order 2N-storage Runge-Kutta driver
"""
