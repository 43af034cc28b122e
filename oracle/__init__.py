"""CPU FP64 oracle for the restarted sketched Krylov f(A)b method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or
executes this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, helpers or constant generators); the only input
both sides consume is the seeded generator package ``workloads``.

Contents (each function cites the passage of the paper it follows):

* ``philox`` / ``sketch`` -- the sparse-sign embedding S (eq. sparse_sign_sketch)
  generated from the counter-based Philox4x32 generator (Salmon et al. 2011), 7 rounds,
  rows drawn without replacement by Floyd's sampling algorithm;
* ``matfun``   -- dense matrix functions (Pade-13 scaling and squaring for exp,
  Schur square root for z^(-1/2)), used for small and growing matrices;
* ``quadrature`` -- partial-fraction rules r(z) = sum_l w_l/(zeta_l - z)
  approximating exp(-t z) (parabolic Hankel contour) and z^(-1/2)
  (Stieltjes integral, tangent substitution);
* ``exact``    -- f(A)b in closed form for the Kronecker-sum test operators
  (sine eigenbasis; Kronecker product of 1-D exponentials) and dense f(A)b;
* ``krylov``   -- unrestarted Arnoldi, plain restarted Arnoldi, and the
  step-by-step twin of the sketched, window-truncated, whitened, restarted
  iteration with both restart evaluations (growing block matrix and
  quadrature recursion).

Parity status of every function is listed in its docstring; all are pinned
by ``tests/test_oracle_*.py`` except where a docstring says "parity unpinned".
"""
from . import philox, sketch, matfun, quadrature, exact, krylov  # noqa: F401
