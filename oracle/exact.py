"""Exact f(A) b for the test operators (the plain result the method converges to).

All test operators are Kronecker sums  A = sum_d I (x) .. (x) T_d (x) .. (x) I + sigma I
of one-dimensional tridiagonal factors T_d on an N-point interior grid with
h = 1/(N+1) (x is the fastest index).  The factors are rebuilt here from the
operator definitions, independently of the CSR assembly in ``workloads``.

* ``sine_fab`` (symmetric factors T_d = c_d h^-2 tridiag(-1, 2, -1)): the
  eigenvectors are Phi_pq = sqrt(2/(N+1)) sin(p q pi/(N+1)) and the
  eigenvalues lambda_p = 4 h^-2 sin^2(p pi / (2(N+1))), so
  f(A) b = Phi^{(x)D} diag(f(sum_d c_d lambda_{p_d} + sigma)) Phi^{(x)D} b,
  applied as D mode products with the symmetric orthogonal Phi.
* ``kron_exp_fab`` (any factors, including non-symmetric convection):
  exp(-t A) = e^{-t sigma} exp(-t T_z) (x) exp(-t T_y) (x) exp(-t T_x); each
  factor is a dense N x N exponential (``matfun.expm``).  ``transpose=True``
  applies exp(-t A^T), the adjoint.
* ``dense_fab`` (tiny n): f of the assembled dense matrix.

Pinned in ``tests/test_oracle_exact.py``: sine basis against the eigen-equation
and dense exp/invsqrt; Kronecker form against dense exp of the assembled
non-symmetric operator.
"""
import numpy as np

from . import matfun


def laplace_factor(N: int, coef: float = 1.0) -> np.ndarray:
    h = 1.0 / (N + 1)
    return coef / h ** 2 * (2.0 * np.eye(N) - np.eye(N, k=1) - np.eye(N, k=-1))


def convdiff_factor(N: int, peclet: float) -> np.ndarray:
    """-d_xx + Pe d_x, central differences: u[i+1] gets -1/h^2 + Pe/(2h), u[i-1] gets -1/h^2 - Pe/(2h)."""
    h = 1.0 / (N + 1)
    return laplace_factor(N) + peclet / (2.0 * h) * (np.eye(N, k=1) - np.eye(N, k=-1))


def sine_basis(N: int):
    p = np.arange(1, N + 1)
    Phi = np.sqrt(2.0 / (N + 1)) * np.sin(np.outer(p, p) * np.pi / (N + 1))
    lam = 4.0 * (N + 1) ** 2 * np.sin(p * np.pi / (2 * (N + 1))) ** 2
    return Phi, lam


def _mode_apply(mats, x: np.ndarray, N: int) -> np.ndarray:
    """Apply mats[d] along axis d (d=0 is x, the fastest index) of the N^D tensor x."""
    D = len(mats)
    T = x.reshape((N,) * D)          # C order: axis D-1 is x
    for d, M in enumerate(mats):
        ax = D - 1 - d
        T = np.moveaxis(np.tensordot(M, T, axes=([1], [ax])), 0, ax)
    return T.reshape(-1)


def sine_fab(fun, b: np.ndarray, N: int, coefs, shift: float = 0.0, t: float = 1.0) -> np.ndarray:
    """f(A) b for A = sum_d coefs[d] * Lap_1D (+) ... + shift I via the sine eigenbasis."""
    D = len(coefs)
    Phi, lam = sine_basis(N)
    y = _mode_apply([Phi] * D, np.asarray(b, dtype=np.float64), N)
    ev = np.zeros((N,) * D)
    for d, c in enumerate(coefs):
        shape = [1] * D
        shape[D - 1 - d] = N
        ev = ev + c * lam.reshape(shape)
    ev = ev + shift
    y = y * matfun.scalar(fun, ev.reshape(-1), t)
    return _mode_apply([Phi] * D, y, N)


def kron_exp_fab(b: np.ndarray, factors, t: float, shift: float = 0.0, transpose: bool = False) -> np.ndarray:
    """exp(-t A) b (or exp(-t A^T) b) for A = factors[0] (+) factors[1] (+) ... + shift I."""
    N = factors[0].shape[0]
    E = [matfun.expm(-t * (F.T if transpose else F)) for F in factors]
    return np.exp(-t * shift) * _mode_apply(E, np.asarray(b, dtype=np.float64), N)


def kron_sum_apply(factors, x: np.ndarray, shift: float = 0.0) -> np.ndarray:
    """A x for A = factors[0] (+) factors[1] (+) ... + shift I (each factor along its own axis)."""
    N = factors[0].shape[0]
    D = len(factors)
    eye = np.eye(N)
    y = shift * np.asarray(x, dtype=np.float64)
    for d, F in enumerate(factors):
        y = y + _mode_apply([F if e == d else eye for e in range(D)], x, N)
    return y


def exp_action_grads(factors, b: np.ndarray, c: np.ndarray, t: float, shift: float = 0.0):
    """L = <c, exp(-t A) b> and its derivatives, from the adjoint identity <c, f(A) b> =
    <f(A^T) c, b> (so dL/db = exp(-t A^T) c) and d/dt exp(-t A) = -A exp(-t A) (so
    dL/dt = -<c, A exp(-t A) b>).  Returns (L, dL/db, dL/dt)."""
    x = kron_exp_fab(b, factors, t, shift)
    L = float(np.dot(c, x))
    gb = kron_exp_fab(c, factors, t, shift, transpose=True)
    gt = -float(np.dot(c, kron_sum_apply(factors, x, shift)))
    return L, gb, gt


def assemble_dense(factors, shift: float = 0.0) -> np.ndarray:
    """The dense Kronecker sum (tiny sizes only)."""
    N = factors[0].shape[0]
    D = len(factors)
    n = N ** D
    A = shift * np.eye(n)
    for d, F in enumerate(factors):
        K = np.ones((1, 1))
        for e in reversed(range(D)):     # slowest axis first
            K = np.kron(K, F if e == d else np.eye(N))
        A = A + K
    return A


def dense_fab(fun, A: np.ndarray, b: np.ndarray, t: float = 1.0) -> np.ndarray:
    return matfun.apply(fun, np.asarray(A, dtype=np.float64), t) @ b


def problem_factors(kind: str, N: int, **kw):
    """(factors, shift) of the named test operator, built from its definition."""
    if kind == "laplacian_2d":
        return [laplace_factor(N)] * 2, 0.0
    if kind == "anisotropic_2d":
        return [laplace_factor(N), laplace_factor(N, kw.get("cy", 0.01))], 0.0
    if kind == "convdiff_3d":
        return [convdiff_factor(N, kw["peclet"])] * 3, 0.0
    if kind == "shifted_laplacian_3d":
        return [laplace_factor(N)] * 3, kw.get("shift", 1.0)
    raise ValueError(kind)
