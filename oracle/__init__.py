"""Plain FP64 CPU oracle for the staggered space-time DG scheme for linear
elasticity (Tavelli & Dumbser, arXiv:1802.04516).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The
product library never calls it and shares no code with it: the two meet only
through the seeded input arrays of ``synth``.

The oracle computes the plain definition of one time slab: it assembles the
coupled velocity-stress slab system of eqs. (NM25)-(NM26) (Section 4), or
its Crank-Nicolson form (NM25.cn)-(NM26.cn), as one sparse matrix and
solves it with a sparse direct LU.  It also forms the explicit velocity
Schur complement of eq. (velocity.sys) / (velocity.sys.cn) for operator
parity and for the symmetry / positive-definiteness theorems of Section 5.1.

Modules
  quad      exact quadrature on simplices (collapsed Gauss-Jacobi)
  basis     nodal P_p velocity basis, Gauss-Legendre-Lagrange time basis,
            raw and canonical dual (stress) bases
  mesh      topology (faces, left/right elements) and geometry
  assemble  the blocks of eqs. (MD_2)-(MD_6)
  slab      coupled slab system, Schur complement, time stepping, energy
  waves     plane-wave exact solutions of Section 6.2 and L2 projections
"""
