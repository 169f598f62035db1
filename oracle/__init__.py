"""FP64 CPU oracle for the EDF-based MesoFD / MMFD explicit time step.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  It shares no code
with the GPU library (``paper_2505_17057_amd``) and never imports it.

* ``oracle.native``  -- ctypes binding of ``mfd_oracle.c`` (whole-grid FP64 steps:
  literal, MesoFD, MMFD, theta; moments; EDF; compensated sums).
* ``oracle.scheme``  -- the host-side algebra of the method (coefficient
  moments, the constraint solve of Eq. (X), presets, PDE-coefficient mapping,
  stability conditions and Fourier amplification).
"""
