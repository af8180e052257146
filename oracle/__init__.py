"""CPU oracle for the FEM-NFFT fast summation -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import
this package.  The product library never imports, links or executes it, and
it imports nothing from the product package.

  oracle.direct   O1: plain FP64 direct sum (C + OpenMP) of the paper's eq. (2)
                  and of H = -grad phi, plus the exact transposes.
  oracle.fastsum  O2: the fast summation's steps in FP64 numpy, in the order the
                  paper's NFFT section describes them (spread with a window,
                  FFT, divide by the window's coefficients) completed by the
                  kernel multiply, inverse transform, gather and near-field
                  correction that the regularized-kernel method needs.
  oracle.fem      the FEM front: quadrature points, weights, charges from a P1
                  magnetization (the paper's eq. (2) and the bullet list after
                  it), the transpose of that charge map, lumped nodal mass and
                  the demagnetizing energy and its exact gradient.
"""
from . import direct, fastsum, fem  # noqa: F401
