"""Plain FP64 CPU oracle of the implicit modal DG solver.

TEST INFRASTRUCTURE ONLY.  Nothing here is part of the product: only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark may
import it.  It shares no code with the HIP library and imports nothing from
the product package.

Franciolini, Fidkowski, Crivellini, "Efficient discontinuous Galerkin
implementations and preconditioners for implicit unsteady compressible flow
simulations" (arXiv 1812.04789):

  reference.py  modal basis and quadrature            (Sec. 3, Eq. BSpace)
  mesh.py       periodic hexahedral mesh and Q1 maps  (Sec. 3)
  physics.py    Euler/NS fluxes, Roe flux             (Sec. 2, Eq. NS; Sec. 3.1)
  dg.py         DG residual with BR2, mass matrix     (Sec. 3.1, Eqs. dg_ns, visc_flux, re)
  linear.py     J.v, block Jacobi, p-multigrid (V-cycle and full multigrid, block-Jacobi or GMRES(BJ)
                smoothers), block ILU(0) in minimum-discarded-fill order, FGMRES
                                                       (Sec. 5.1 Eq. DG-mf; Sec. 6, Alg. 1, Alg. 2; Sec. 6.1;
                                                        Sec. 6.3; Table MGSettings)
  timestep.py   BDF2 and ESDIRK3 steps with Newton     (Sec. 4, Eq. NEWTON)

Every function is written from the equations, vectorised over elements with
dense reference matrices (no sum factorisation, no fused kernels), so it can
be checked against the paper by eye.
"""
