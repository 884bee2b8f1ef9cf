"""CPU FP64 oracle for the matrix-free (Navier-)Stokes hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The HIP library
never calls it, and it shares no code with the HIP library: the two meet only
in the seeded inputs of ``inputs/``.

What it computes is the plain definition of each operation of the paper
(Munch et al., "Solving the (Navier-)Stokes equations with space and time
adaptivity using deal.II"):

* element matrices by full Gauss quadrature over the tensor-product Lagrange
  basis with no sum factorisation, assembled into sparse matrices
  (Sec. 1, eq. (stokes) and (ns); Sec. 3, eq. (stokes_block));
* the cell-wise transfer of Sec. 2, eq. (transfer), as an assembled sparse
  matrix;
* Chebyshev smoothing, the multigrid V-cycle, the Silvester-Wathen block
  preconditioner, PCG and FGMRES (Sec. 2 and 3) step by step with those
  matrices;
* the SUPG/PSPG stabilised Navier-Stokes residual and its Jacobian (Sec. 5).

Readings of the paper where it is silent are listed in each module header.
Functions whose result has no independent pin say "parity unpinned".
"""
