"""MI355X-native Fourier pseudo-spectral Navier--Stokes time integrator.

Importing the package loads nothing native; the HIP library is loaded on
first use of :mod:`paper_1810_10197_amd.ns` (which raises if it is missing).
"""
