"""FP64 CPU oracle for the recursive-regularised lattice Boltzmann update.

TEST INFRASTRUCTURE ONLY. Nothing in the product path (the HIP library, its
Python binding) imports, calls or links anything in this package; only the
tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code, table or constant generator with the
GPU path: its lattice tables come from a Gauss--Hermite rule and a moment
solve, its collision is the dense Hermite projection ``f = W H^T G^-1 a`` and
its off-equilibrium coefficients come from the paper's recursion applied to
index tuples, whereas the GPU path uses unrolled tensor-product register code
and the pair-sum closed form.

Modules
  lattice      velocity sets, weights, Hermite basis, Gram matrices
               (Sec. 3.2, "Discretization of the microscopic velocity space")
  rr           moments, equilibrium / off-equilibrium Hermite coefficients,
               regularised collision and periodic streaming (Secs. 2, 3.1,
               3.4, 3.5; App. A/B)
  lsa          von Neumann linear stability analysis of the collision
               (Sec. 3.6)
  diagnostics  global mass / momentum / kinetic energy / enstrophy
               (Sec. 4.1 energy and enstrophy definitions)
  mlp          FP64 reference of the learned-closure MLP with BF16 rounding
               points replicated (no counterpart in the paper)

All arithmetic is IEEE binary64 (numpy), no fast-math, unless a function says
otherwise.  Array layout: populations ``f[i, z, y, x]`` (x fastest), velocity
``u[d, z, y, x]``; 2D lattices use nz = 1.
"""
