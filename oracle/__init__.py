"""Reference oracle for the conservative cut-cell Navier-Stokes method.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow FP64 CPU statement of
what the method computes, written from the paper (Quiros Rodriguez, Fullana,
Le Chenadec, Sayadi, "A Conservative Cartesian Cut Cell Method for the
Solution of the Incompressible Navier-Stokes Equations on Staggered Meshes").
Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import it.  The device library never calls it and shares no code with it.

Modules
  levelset   level-set functions of the synthetic bodies
  geometry   capacities of the first and second kind (Sec. 3.2-3.4)
  calculus   unit-spacing difference, midpoint interpolation, permanent product
  operators  cont, pres, strain, visc, conv, kinetic (Sec. 4.1-4.5)
  derived    activity masks and coefficient fields used by the time stepper
  solvers    Jacobi-preconditioned CG and a direct sparse solve
  pmii       projection method II time step (Sec. 4.6)
  geometry3d capacities of the first kind in three dimensions (spheres and
             z-cylinders; Sec. 3.2-3.4 with a third index)
  pmii3d     the projection step in three dimensions (Sec. 4.1, 4.6)

Parity status: every function is pinned by a test under tests/ except the
ones whose header says "parity unpinned".
"""
