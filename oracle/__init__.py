"""CPU FP64 oracle for accelerated cyclic reduction (test infrastructure only).

This package is the slow, plain reference the GPU library is checked against.
Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import it; the GPU library never does, and the two share no code.  Everything
here is dense numpy/scipy in float64:

* ``cluster``  - planar bisection cluster tree and the red/black level schedule
  (Sections 2.1.1, 2.2.2, 3.1; Eq. permuted_system).
* ``hodlr``    - block-wise truncation T(.) of a dense plane block to the
  weak-admissibility (HODLR) format (Sections 2.1, 2.1.1, 3.1).
* ``acr``      - block cyclic reduction with T(.) after every block operation
  (Eq. elim, Algorithms 1 and 2), its back-substitution (Eq. all_backSubs) and
  the transpose solve that reuses the same blocks.
* ``assemble`` - an independent sparse assembly of the model operators and the
  relative residual of Section 5.
* ``gradient`` - loss and adjoint gradient with respect to the per-node
  diffusion coefficient.

Parity status: every function is pinned by a CPU test against closed forms,
library solvers or brute force (see tests/test_oracle_*.py), except the
truncated (eps > 0) factorisation, whose exact values admit several correct
results; there the pins are bounds (Eckart-Young per block, residual <= C*eps)
and the transpose identity, and element values are "parity unpinned".
"""
