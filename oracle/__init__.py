"""FP64 CPU oracle for the FFT-based binned bispectrum estimator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the tests, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the HIP path.

Modules
  geometry  shells, triangle selection, bin labels (Section 2.1, eqs. cond, shape)
  fbe       the fast estimator in float64 (Section 2.2, eqs. kdelta, bsfin, iFT, Ntri2, 2FT)
  dbe       the direct triple sum over closed mode triangles (eqs. binbs, Ntri1)
  adjoint   gradient of a linear functional of B with respect to delta(x)
  analytic  tree-level B of the quadratic non-Gaussian field (eq. bana) and the
            linear-RSD monopole (eq. RSD)
  polyspectrum  the fourth-order polyspectrum estimator (Section 4: four shell
            fields, cutoff 2 pi N_g / (4 L)) and its closed-4-tuple sum
  multipoles  Legendre moments (l = 0, 2, 4) of the redshift-space bispectrum
            in the angle of the first side to the line of sight (Section 3.1)
            and their weighted closed-triangle sum
"""
