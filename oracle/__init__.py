"""Plain FP64 CPU oracle for the randomized SVD hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or link anything in this package; only the
tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
use it.  It shares no code, tables or constants generator with the HIP path.

Every function is written to be checked against the paper by eye: it follows
the steps of the randomized SVD (Section 2.1, steps 1-7), the power matrix
(Section 2.2, Eqs. (1)-(2)) and the block-wise product / block-cyclic layout
(Section 2.3, Eq. (3); Section 3.1), in FP64 throughout, with no blocking,
fusion or reordering beyond what those passages state.

Modules
  philox      counter-based Philox-4xW-10 generator and the Gaussian test
              matrix built from it (Section 2.1, step 1)
  householder thin Householder QR (Section 2.1, steps 3-4)
  jacobi      one-sided Jacobi SVD and cyclic Jacobi symmetric eigensolver
              (Section 2.1, step 6)
  rsvd        the randomized SVD with power iteration (Sections 2.1-2.2)
  tilemap     block-cyclic tile maps and visit orders (Sections 2.3, 3.1)
  adjoint     the truncated-SVD adjoint used for the backward pass
  metrics     sigma error, subspace angle and residual measures
  storage     storage accounting of matrices and factors

Parity status of each function is stated in its module header.
"""

from . import philox, householder, jacobi, rsvd, tilemap, metrics, adjoint, storage  # noqa: F401
