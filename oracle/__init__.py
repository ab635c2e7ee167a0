"""CPU FP64 oracle for the S_N upwind-DG source iteration with synthetic acceleration.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import, call, link or run anything in this package.
The GPU library and its binding never import it and share no code with it.

Contents (each function cites the paper passage it follows):
  quadrature  normalized angular rules (Sec. 2.1)
  dg          upwind-DG element operators by Gauss quadrature (Sec. 2.2)
  csweep.c    plain C transport sweeps (Sec. 2.3, eq. (transport_sweep))
  problem     discretized single instances (eq. (dg_matrix_vec))
  sisa        Alg. 1 (SI / SI-DSA / ROMSA / ROMSAD with Alg. 2)
  dsa         consistent slab DSA (Appendix B); MIP diffusion form in 2D (reading)
  rom         POD correction ROM, ROMSA, parametric ROM / ROMIG (Sec. 3)
  brute       dense global solve of eq. (one_equation), ideal correction
"""
