"""FP64 CPU oracle for the P^T N^-1 P map-making path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the test suite, the package smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP path
(no kernels, headers, helpers, tables or constant generators); the only thing
both sides share is the seeded input data made by the synthetic workload
generator, which holds none of the method's arithmetic.

Everything here is plain, slow, obviously-correct NumPy in float64, written
to be checked against the paper by eye:

  healpix    HEALPix ring-scheme ang2pix / pix2ang (the sky discretisation of
             the "Landscape types" paragraph, section "Software Design").
  pointing   the pointing operator P and its transpose (IndexOperator,
             PointingOperator, QURotationOperator, HWPOperator,
             LinearPolarizerOperator of Tables 2 and 3; rotation merging and
             the HWP commutation rule of "Algebraic reductions").
  noise      N^-1: diagonal (HomothetyOperator / DiagonalOperator) and
             symmetric band-Toeplitz (SymmetricBandToeplitzOperator, Table 2)
             by direct summation, dense matrix and FFT linear convolution.
  mapmaker   the GLS / maximum-likelihood estimator of Eq. (2) with the
             block-Jacobi preconditioner ("Map-making classes") solved by
             preconditioned conjugate gradients (the inverse "A.I(solver=...,
             preconditioner=...)" of Table 1).
  chi2       chi-square of the data model of Eq. (1) and its analytic
             gradient with respect to the map, detector gains and
             polarisation-angle offsets (differentiability, "Summary" and
             "Research Impact Statement").

Parity status of each function is stated in its module header.
"""
from . import healpix, pointing, noise, mapmaker, chi2  # noqa: F401
