"""Oracle: plain, slow, serial CPU implementation of the partitioned P-ERK + DGSEM method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or runs any file
in this directory; only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may use it.  It shares no code with the HIP path: its own mesh connectivity,
quadrature, fluxes, mortar operators, Runge-Kutta tableaux and partition rule.

Modules
  perk_coeffs  P-ERK tableaux from stability polynomials (Sec. 3.1, 4.3), order conditions
               (Sec. 2.1), stability polynomial of a tableau, LP optimiser (Sec. 4.2).
  godunov1d    1D first-order Godunov advection + partitioned RK (Sec. 3.2.1-3.2.5).
  dgsem        ctypes wrapper of dgsem.cpp: DGSEM for 2D/3D Euler and Navier-Stokes (BR1)
               on a Cartesian forest with 2:1 mortars, the dense masked partitioned RK step
               (Sec. 2, eq. PartitionedRKSystem) and AMR helpers.

Floating point is fp64 throughout (the paper works in standard double precision, Sec. 4.2).
"""
