"""CPU FP64 oracle for the homogeneous-medium RTE Fredholm solver.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import or run anything in this package; the product path (the HIP library and its
Python binding) never does, and shares no code with it.

What it computes is the plain definition of the discrete problem of Fan, An and Ying,
"Fast algorithms for integral formulations of steady-state radiative transfer equation":

  (I - K~ D) u = K~ g,   u in C^{N M},  g_{j,k} = f(x_j) delta_{k0},  D = diag_k(mu_s sigma_hat_k)

(eq. ani_AU, Sec. 3.3; eq. iso_AU with the u-form of eq. iso_Fredholm, Sec. 2.3), with the
Nystrom matrix K~ of eq. ani_discretization: point values of the kernel times the cell volume
off the diagonal and the exact cell integral of the singular kernel on the diagonal.

Modules
  kernels     kernel entries, exact self-cell integrals (2D modes, 3D isotropic)
  operator2d  dense matrix, direct-sum apply, sampled apply, FFT apply (2D, 2L+1 modes)
  operator3d  the same for the 3D isotropic kernel
  krylov      dense LU, unrestarted GMRES, Neumann series
  scattering  the scattering term S(x, theta) at discrete angles from the modes (eq. ani_2d_scattering)
  closed_form the mu_s = 0 solution for f = 1 on the unit square/cube (attenuated source)
  convnet     3x3 convolution network forward/backward in FP64 (learned preconditioner)

Readings of passages the paper leaves ambiguous are stated where they are used (self-cell
weight, angle convention, sign of the mode exponent, padding, Krylov details).
"""
