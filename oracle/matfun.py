"""Dense matrix functions for small and growing matrices (FP64).

* ``expm``: scaling and squaring with the diagonal [13/13] Pade approximant
  (Higham 2005, the method the paper's appendix names for exp and phi_1).  The
  Pade coefficients are computed from their closed form
  c_j = (2p-j)! p! / ((2p)! j! (p-j)!), p = 13, not typed in.  Only the
  degree-13 branch is used (more flops for small norms, same accuracy).
* ``invsqrt``: z^(-1/2) through the Schur-method principal square root
  (scipy.linalg.sqrtm) followed by a linear solve; used where the paper's
  restart needs f of a non-normal matrix (reading: Schur-based evaluation,
  because an eigendecomposition is unstable on the growing restart matrix).
* ``apply``: dispatch by function name.

Pinned in ``tests/test_oracle_matfun.py`` against closed forms (rotation
generators, nilpotent and diagonal matrices) and against scipy.
"""
from fractions import Fraction
from math import factorial

import numpy as np
import scipy.linalg as sla

_P = 13
_C = [Fraction(factorial(2 * _P - j) * factorial(_P), factorial(2 * _P) * factorial(j) * factorial(_P - j))
      for j in range(_P + 1)]
PADE13 = np.array([float(c) for c in _C])
THETA13 = 5.371920351148152   # Higham (2005), Table 2.3: 1-norm bound for degree 13


def expm(A: np.ndarray) -> np.ndarray:
    A = np.asarray(A)
    n = A.shape[0]
    nrm = np.linalg.norm(A, 1)
    s = 0 if nrm <= THETA13 else int(np.ceil(np.log2(nrm / THETA13)))
    A = A / (2.0 ** s)
    b = PADE13
    I = np.eye(n, dtype=A.dtype)
    A2 = A @ A
    A4 = A2 @ A2
    A6 = A4 @ A2
    U = A @ (A6 @ (b[13] * A6 + b[11] * A4 + b[9] * A2) + b[7] * A6 + b[5] * A4 + b[3] * A2 + b[1] * I)
    V = A6 @ (b[12] * A6 + b[10] * A4 + b[8] * A2) + b[6] * A6 + b[4] * A4 + b[2] * A2 + b[0] * I
    R = np.linalg.solve(V - U, V + U)
    for _ in range(s):
        R = R @ R
    return R


def invsqrt(A: np.ndarray) -> np.ndarray:
    Z = sla.sqrtm(np.asarray(A, dtype=complex if np.iscomplexobj(A) else float))
    Y = np.linalg.solve(Z, np.eye(A.shape[0]))
    if not np.iscomplexobj(A):
        Y = Y.real if np.abs(Y.imag).max() <= 1e-12 * np.abs(Y).max() else Y
    return Y


def apply(fun: str, A: np.ndarray, t: float = 1.0) -> np.ndarray:
    """f(A) for fun in {"exp" (exp(-t A)), "invsqrt" (A^(-1/2))}; callables are applied as f(A)."""
    if callable(fun):
        return fun(A)
    if fun == "exp":
        return expm(-t * np.asarray(A))
    if fun == "invsqrt":
        return invsqrt(A)
    raise ValueError(fun)


def scalar(fun, z, t: float = 1.0):
    """The same function on scalars (used by closed-form oracles)."""
    if callable(fun):
        return fun(z)
    if fun == "exp":
        return np.exp(-t * z)
    if fun == "invsqrt":
        return 1.0 / np.sqrt(z)
    raise ValueError(fun)
