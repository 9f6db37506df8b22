"""CPU FP64 oracle for the assembly-free deflated voxel solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path (its own element matrix, indexing, assembly and solvers).

It computes the plain definitions the method reaches:

* the static equilibrium ``K u = f`` of the finite element model (Eq. 1.1),
  with K assembled globally from per-element matrices and solved directly or
  by textbook (deflated) conjugate gradients on the assembled matrix;
* the compliance ``J = f . u`` (Eq. 1.3-1.4);
* the per-element strain-energy sensitivity ``s_e = rho_e u_e^T Ke u_e``, the
  element-sensitivity route of Sec. 3.1 (the element term of Eq. 3.5);
* the topology extracted from a sensitivity field at a volume fraction
  (Eq. 3.6 with the cutting value set by the target volume, Sec. 3.2).

Modules: ``fem`` (element matrix, mesh indexing, assembly), ``solvers``
(direct, Jacobi-PCG, deflated PCG), ``post`` (compliance, sensitivity, ranking),
``casting`` (the casting projection of Sec. 3.7), ``levelset`` (the augmented
topological level-set loop of Sec. 3.2-3.4 and 3.8 on direct solves),
``stress`` (the p-norm von Mises stress, its adjoint and field, Eq. 3.3),
``modal`` (mass matrix, lowest eigenpairs and their sensitivity, Eq. 3.4),
``buckling`` (geometric stiffness, load factors and their sensitivity, Eq. 3.5).
"""
from . import fem, solvers, post  # noqa: F401
