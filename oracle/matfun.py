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
* ``phi1``: phi_1(M) = (e^M - I) M^{-1} (the phi function of eq. conv_diff_sol3)
  without inverting M, through the augmented exponential
  exp([[M, I], [0, 0]]) = [[e^M, phi_1(M)], [0, I]] (the block of the
  exponential of a block upper-triangular matrix: the integral
  int_0^1 e^{sM} ds = phi_1(M)); the same Pade-13 scaling and squaring.
* ``cos_sqrt``: cos(t sqrt(A)) (the membrane solution of eq. drum_sol) without
  a square root, through the first-order form of u'' = -A u:
  exp(t [[0, I], [-A, 0]]) = [[cos(t sqrt A), .], [., cos(t sqrt A)]]; the
  series of cos(t sqrt z) has only integer powers of z, so any square root of
  A gives the same matrix (as the paper notes for eq. drum_sol).
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


def phi1(M: np.ndarray) -> np.ndarray:
    """phi_1(M) = sum_k M^k / (k+1)!, the top-right block of exp([[M, I], [0, 0]])."""
    M = np.asarray(M)
    n = M.shape[0]
    B = np.zeros((2 * n, 2 * n), dtype=M.dtype)
    B[:n, :n] = M
    B[:n, n:] = np.eye(n)
    return expm(B)[:n, n:]


def cos_sqrt(A: np.ndarray, t: float = 1.0) -> np.ndarray:
    """cos(t sqrt(A)) = sum_k (-t^2 A)^k / (2k)!, the top-left block of exp(t [[0, I], [-A, 0]])."""
    A = np.asarray(A)
    n = A.shape[0]
    B = np.zeros((2 * n, 2 * n), dtype=A.dtype)
    B[:n, n:] = t * np.eye(n)
    B[n:, :n] = -t * A
    return expm(B)[:n, :n]


def apply(fun: str, A: np.ndarray, t: float = 1.0) -> np.ndarray:
    """f(A) for fun in {"exp" (exp(-t A)), "invsqrt" (A^(-1/2)), "phi1" (phi_1(-t A)),
    "cos_sqrt" (cos(t sqrt(A)))}; callables are applied as f(A)."""
    if callable(fun):
        return fun(A)
    if fun == "exp":
        return expm(-t * np.asarray(A))
    if fun == "invsqrt":
        return invsqrt(A)
    if fun == "phi1":
        return phi1(-t * np.asarray(A))
    if fun == "cos_sqrt":
        return cos_sqrt(A, t)
    raise ValueError(fun)


def scalar(fun, z, t: float = 1.0):
    """The same function on scalars (used by closed-form oracles and the rule checks)."""
    if callable(fun):
        return fun(z)
    if fun == "exp":
        return np.exp(-t * z)
    if fun == "invsqrt":
        return 1.0 / np.sqrt(z)
    if fun == "phi1":  # phi_1(-t z) = (1 - e^{-t z}) / (t z), 1 at z = 0
        s = -t * np.asarray(z)
        small = np.abs(s) < 1e-8
        safe = np.where(small, 1.0, s)
        return np.where(small, 1.0 + s / 2.0, np.expm1(safe) / safe)
    if fun == "cos_sqrt":  # cos(t sqrt(z)); for z < 0 this is cosh(t sqrt(-z))
        z = np.asarray(z)
        v = np.cos(t * np.sqrt(z.astype(complex)))
        return v.real if not np.iscomplexobj(z) else v
    raise ValueError(fun)
