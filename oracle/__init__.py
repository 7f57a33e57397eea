"""CPU FP64 oracle for the Fourier pseudo-spectral Navier--Stokes time integrator.

TEST INFRASTRUCTURE ONLY.  This package is a deliberately plain, slow and
obviously correct NumPy implementation of what the GPU path computes, written
from Ketcheson, Mortensen, Parsani & Schilling, "More efficient time
integration for Fourier pseudo-spectral DNS of incompressible turbulence"
(arXiv:1810.10197).  Only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import it; the product path never does, and it shares
no code with the HIP library (no kernels, headers, tables or helpers).

Conventions used throughout (readings of the paper where it is silent or
garbled):

* grid x_j = 2*pi*j/N on [0, 2*pi)^d, physical arrays indexed [z][y][x]
  (3D) or [y][x] (2D), x contiguous;
* spectral arrays are the half spectrum of ``numpy.fft.rfftn`` over the
  spatial axes, indexed [kz][ky][kx] (3D) or [ky][kx] (2D), kx = 0..N/2;
* normalised transform: u_hat = DFT(u) / N^d, so physical values are
  recovered by ``irfftn(u_hat * N^d)``;
* 2/3-rule dealiasing: a mode is retained iff |k_j| <= K = (N-1)//3 on every
  axis.

Modules
-------
spectral     wavenumbers, mask, naive DFT, RHS of Eq. (2) and Eqs. (4a-b)
tableaux     RK4, BS5 and DP5 coefficients as exact rationals (Appendix A)
stepping     one RK4 step, one BS5 attempt with the embedded error (Sec. 2.2)
control      step-size controller and the adaptive integrate loop (Sec. 2.2.1)
diagnostics  kinetic energy, dissipation rate, shell spectrum (Sec. 3.1)
forcing      post-step low-wavenumber rescale for HIT (Sec. 3.3.1)
mlp          20-64-64-1 tanh step-size proposer: forward, backward, Adam
"""
