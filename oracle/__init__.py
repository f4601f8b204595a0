"""Plain CPU oracle for the dual-primal spectral-element Helmholtz method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or execute this package; only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use it.

It follows Galagusz & McFee, "An iterative domain decomposition, spectral
finite element method on non-conforming meshes suitable for high frequency
Helmholtz problems" (arXiv:1808.04713), in complex128 with NumPy/SciPy,
step by step and without blocking or fusion:

  legendre   -- 1-D Legendre toolkit (Sec. 2.1.1, 2.1.6)
  element    -- element matrices and loads (Sec. 2.1.5, 2.2.1)
  mesh       -- quadtree leaves, neighbours, affine parameters (Sec. 2.2.3-2.2.4)
  constraints-- hierarchical moment constraints and Algorithm 1 (Sec. 2.2.4, 2.3.2)
  dp         -- literal partial-nullspace dual-primal method (Sec. 2.3.1-2.3.4)
  dp_elementwise -- the same method written element by element (Sec. 2.3.3)
  dp_nonconforming -- element by element on quadtree meshes with hanging edges
                (Sec. 2.2.4, 2.3.1-2.3.3; basis of the kept modes)
  independent -- saddle-point sparse LU and a nodal C0 spectral-element solve
  adjoint    -- far-field intensity and its permittivity gradient by an adjoint solve
  direct     -- globally conforming Galerkin solution by a direct solve
  gmres      -- left-preconditioned GMRES (Sec. 2.3.4, 3.2)
  farfield   -- far-field integral and RCS (Sec. 3.3.1)
"""
