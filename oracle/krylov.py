"""Krylov twins of the method, in plain FP64 numpy/scipy (test infrastructure).

Notation follows the paper: basis W, sketch U = S W, upper Hessenberg R
(Alg. 1); whitening factor T from the thin QR of S W (appendix, eq. A.1);
cycles of Alg. 2.

One cycle from a start vector v (reading of the path; k-window truncation of
Alg. 1, whitening of eq. A.1, quadrature restart of Section 4):

    alpha = ||S v||, w_1 = v/alpha, u_1 = S v/alpha                  (Alg. 1)
    for j = 1..m:  z = A w_j, u = S z
        for i = max(1, j-k+1)..j:  r_ij = <u_i, u>, u -= r_ij u_i   (modified GS, sketch space)
        rho = ||u||; w_{j+1} = (z - sum_i r_ij w_i)/rho; u_{j+1} = u/rho
    U_{m+1} = Q T_{m+1},  T_{m+1} = [[T_m, t], [0, tau]],  diag(T) > 0
    X = T_m R_m T_m^{-1} + (r_{m+1,m}/T_m[m,m]) t e_m^T,   h = r_{m+1,m} tau / T_m[m,m]
    V = W_m T_m^{-1},  v_hat = (w_{m+1} - V t)/tau,  beta = alpha T[1,1]

so that A V = V X + h v_hat e_m^T (an Arnoldi-like decomposition, eq.
rand_arnoldi) and v = beta V e_1.  Stacking cycles gives the block lower
bidiagonal matrix M_c with diagonal blocks X^(i) and coupling blocks
h^(i) beta^(i+1) e_1 e_m^T (eq. restart_combined with R -> X), and the
approximation f_c = beta^(1) [V^(1) .. V^(c)] f(M_c) e_1 (eq. restart_approx).
With k >= m the sketch basis is orthonormal, T = I and X = R: the paper's
restart-rand exactly.

Restart evaluations of block c of f(M_c) e_1:

* ``GrowingRestart``: assemble M_c and evaluate f on it densely (Alg. 2,
  F = f(R_km)), as the paper does.
* ``QuadratureRestart``: with r(z) = sum_l w_l/(zeta_l - z), block forward
  substitution of (zeta - M_c) y = e_1 gives block c of r(M_c) e_1 as
  sum_l w_l psi_c(zeta_l) beta_c (zeta_l - X^(c))^{-1} e_1 / beta_1 ... i.e.
  g_c = beta_c sum_l w_l psi_l Y_l,  psi_l <- psi_l beta_c h_c [Y_l]_m,
  Y_l = (zeta_l I - X^(c))^{-1} e_1, psi = 1 at the first cycle.

Stopping (Alg. 2 and the error estimate after it): the difference of two
successive cycles, y_c = V^(c) g_c, continued by the geometric tail of the
increments (``tail_estimate``); stop when that estimate is <= tol ||x_c||.
Breakdown (rho <= 64 eps ||S z||) ends the cycle early with an exact
invariant subspace: f is applied to the leading j x j block and the solve ends.

Pins: tests/test_oracle_krylov.py (polynomial exactness, m >= dim K exactness,
k >= m reduction to T = I, S = I reduction to plain Arnoldi, quadrature vs
growing evaluation, the similarity lemma, closed-form results).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import matfun, quadrature

EPS = np.finfo(np.float64).eps


# ----------------------------------------------------------------------------- cycles
@dataclass
class Cycle:
    """One cycle's basis data in the whitened form A V = V X + h v_hat e_m^T."""
    m: int                  # number of basis vectors used (m, or j at breakdown)
    W: np.ndarray           # n x (m+1) (column m unused at breakdown)
    U: np.ndarray | None    # d x (m+1) sketch S W (None for plain Arnoldi)
    R: np.ndarray           # (m+1) x m upper Hessenberg
    alpha: float
    T: np.ndarray           # (m+1) x (m+1) (m x m at breakdown) upper triangular, diag > 0
    X: np.ndarray           # m x m
    h: float
    beta: float
    Tinv: np.ndarray        # m x m
    vhat: np.ndarray | None
    breakdown: bool

    def basis_apply(self, g: np.ndarray) -> np.ndarray:
        """V g = W_m (T_m^{-1} g)."""
        return self.W[:, :self.m] @ (self.Tinv @ g)


def randomized_arnoldi_window(A, S, v, m: int, k: int, orth: str = "sketch"):
    """Alg. 1 with the Gram-Schmidt loop limited to the last k vectors.

    orth="sketch": sketched inner products (randomized Gram-Schmidt of Algorithm 1);
    orth="full":   full-space inner products and 2-norm normalisation (the
                   incomplete orthogonalization of the comparison methods), with
                   U = S W formed afterwards for whitening.
    Returns (W, U, R, alpha, m_eff, breakdown).
    """
    n = v.shape[0]
    d = S.shape[0]
    W = np.zeros((n, m + 1))
    U = np.zeros((d, m + 1))
    R = np.zeros((m + 1, m))
    u = S @ v
    if orth == "sketch":
        alpha = np.linalg.norm(u)
        W[:, 0] = v / alpha
        U[:, 0] = u / alpha
    else:
        alpha = np.linalg.norm(v)
        W[:, 0] = v / alpha
        U[:, 0] = S @ W[:, 0]
    m_eff, brk = m, False
    for j in range(m):
        z = A @ W[:, j]
        lo = max(0, j - k + 1)
        if orth == "sketch":
            u = S @ z
            raw = np.linalg.norm(u)
            for i in range(lo, j + 1):
                R[i, j] = U[:, i] @ u
                u = u - R[i, j] * U[:, i]
            rho = np.linalg.norm(u)
        else:
            wz = z.copy()
            raw = np.linalg.norm(wz)
            for i in range(lo, j + 1):
                R[i, j] = W[:, i] @ wz
                wz = wz - R[i, j] * W[:, i]
            rho = np.linalg.norm(wz)
        if rho <= 64.0 * EPS * raw:
            m_eff, brk = j + 1, True
            break
        R[j + 1, j] = rho
        W[:, j + 1] = (z - W[:, lo:j + 1] @ R[lo:j + 1, j]) / rho
        U[:, j + 1] = (u / rho) if orth == "sketch" else (S @ W[:, j + 1])
    return W, U, R, float(alpha), m_eff, brk


def whiten(W, U, R, alpha, m_eff, brk) -> Cycle:
    """Thin QR of the sketch and the whitened projected matrix (eq. A.1 and its restart form)."""
    m = m_eff
    cols = m if brk else m + 1
    _, T = np.linalg.qr(U[:, :cols], mode="reduced")
    sgn = np.where(np.diag(T) < 0, -1.0, 1.0)
    T = sgn[:, None] * T                      # positive diagonal (appendix: sign of t_11)
    Tm = T[:m, :m]
    Tinv = np.linalg.solve(Tm, np.eye(m))
    Rm = R[:m, :m]
    X = Tm @ Rm @ Tinv
    if brk:
        h, vhat = 0.0, None
    else:
        t, tau, r = T[:m, m], T[m, m], R[m, m - 1]
        X = X + (r / Tm[m - 1, m - 1]) * np.outer(t, np.eye(m)[m - 1])
        h = r * tau / Tm[m - 1, m - 1]
        vhat = (W[:, m] - W[:, :m] @ (Tinv @ t)) / tau
    return Cycle(m, W, U, R, alpha, T, X, float(h), float(alpha * T[0, 0]), Tinv, vhat, brk)


def sketched_cycle(A, S, v, m: int, k: int, orth: str = "sketch") -> Cycle:
    return whiten(*randomized_arnoldi_window(A, S, v, m, k, orth))


def arnoldi_cycle(A, v, m: int) -> Cycle:
    """Classical Arnoldi with two classical Gram-Schmidt passes (CGS2); V orthonormal.

    In the whitened notation T = I, X = H_m, h = h_{m+1,m}, v_hat = v_{m+1},
    beta = ||v|| (the paper's restart, Section 2.2 and the method list).
    """
    n = v.shape[0]
    V = np.zeros((n, m + 1))
    H = np.zeros((m + 1, m))
    beta = np.linalg.norm(v)
    V[:, 0] = v / beta
    m_eff, brk = m, False
    for j in range(m):
        z = A @ V[:, j]
        raw = np.linalg.norm(z)
        for _ in range(2):
            c = V[:, :j + 1].T @ z
            z = z - V[:, :j + 1] @ c
            H[:j + 1, j] += c
        rho = np.linalg.norm(z)
        if rho <= 64.0 * EPS * raw:
            m_eff, brk = j + 1, True
            break
        H[j + 1, j] = rho
        V[:, j + 1] = z / rho
    mm = m_eff
    I = np.eye(mm + (0 if brk else 1))
    return Cycle(mm, V, None, H, float(beta), I, H[:mm, :mm].copy(),
                 0.0 if brk else float(H[mm, mm - 1]), float(beta), np.eye(mm),
                 None if brk else V[:, mm].copy(), brk)


def arnoldi_full(A, b, m: int, fun, t: float = 1.0):
    """Unrestarted Arnoldi approximation f_m = beta V_m f(H_m) e_1 (Section 2.2)."""
    cyc = arnoldi_cycle(A, b, m)
    F = matfun.apply(fun, cyc.X, t)
    return cyc.beta * (cyc.W[:, :cyc.m] @ F[:, 0])


# ----------------------------------------------------------------------------- restarts
class GrowingRestart:
    """Block c of f(M_c) e_1 from the explicitly assembled growing matrix (Alg. 2)."""

    def __init__(self, fun, t: float = 1.0):
        self.fun, self.t = fun, t
        self.M = np.zeros((0, 0))
        self.beta1 = None
        self.prev_h = None

    def step(self, X: np.ndarray, h: float, beta: float) -> np.ndarray:
        m = X.shape[0]
        p = self.M.shape[0]
        M = np.zeros((p + m, p + m))
        M[:p, :p] = self.M
        M[p:, p:] = X
        if p == 0:
            self.beta1 = beta
        else:
            M[p, p - 1] = self.prev_h * beta
        self.M, self.prev_h = M, h
        F = matfun.apply(self.fun, M, self.t)
        g = self.beta1 * F[p:, 0]
        return g.real if np.iscomplexobj(g) else g


class QuadratureRestart:
    """Block c of r(M_c) e_1 by the recursion over fixed quadrature nodes (fixed m x m work)."""

    def __init__(self, zeta: np.ndarray, w: np.ndarray, half: bool):
        self.zeta, self.w, self.half = np.asarray(zeta, complex), np.asarray(w, complex), half
        self.psi = np.ones(len(self.zeta), dtype=complex)

    def step(self, X: np.ndarray, h: float, beta: float) -> np.ndarray:
        m = X.shape[0]
        e1 = np.zeros(m, dtype=complex)
        e1[0] = 1.0
        acc = np.zeros(m, dtype=complex)
        last = np.zeros(len(self.zeta), dtype=complex)
        for l, z in enumerate(self.zeta):
            y = np.linalg.solve(z * np.eye(m) - X, e1)
            acc += self.w[l] * self.psi[l] * y
            last[l] = y[m - 1]
        self.psi = self.psi * (beta * h) * last
        g = beta * acc
        return 2.0 * g.real if self.half else g.real



def make_rule(fun, t: float = 1.0, n_quad: int | None = None, spec=None):
    """(zeta, w, half) for the named function; see ``quadrature``."""
    if fun == "exp":
        N, P, mu, L = quadrature.EXP_MAIN
        N = n_quad or N
        z, w = quadrature.exp_rule(t, N, P, mu, L)
        z, w = quadrature.conjugate_half(z, w)
        return z, w, True
    if fun == "invsqrt":
        N = n_quad or 128
        z, w = quadrature.invsqrt_rule(N, spec[0], spec[1])
        return z, w, False
    if fun == "phi1":
        N, P, mu, L = quadrature.EXP_MAIN
        z, w = quadrature.phi1_rule(t, n_quad or N, P, mu, L)
        z, w = quadrature.conjugate_half(z, w)
        return z, w, True
    if fun == "cos_sqrt":
        z, w = quadrature.cos_sqrt_rule(t, n_quad or quadrature.COS_SQRT_N, spec[0], spec[1])
        z, w = quadrature.conjugate_half(z, w)
        return z, w, True
    raise ValueError(fun)


# ----------------------------------------------------------------------------- stopping test
UNIT_ROUNDOFF = 2.0 ** -53  # FP64, the oracle's arithmetic


def tail_estimate(ynorm: float, xnorm: float, history: list, unit_roundoff: float = UNIT_ROUNDOFF) -> float:
    """Estimated remaining relative error after a cycle (the stopping test of the restart).

    Section 4 estimates the error of the restarted iterate by the difference of two successive
    cycles, ||y_c|| = ||x_c - x_{c-1}||.  Read as the first term of the remaining increments, which
    a converging restart shrinks by a roughly constant ratio q = ||y_c|| / ||y_{c-1}||, the error
    left after cycle c is the geometric tail ||y_c|| q / (1 - q) (exact when every increment is
    the previous one times q).  q is the largest of the last TAIL_RATIOS ratios (fewer in the first
    cycles), so small ratios between growing increments (a dip in a transient) do not end the loop;
    with q >= 1, or after the first cycle (no ratio yet), the estimate is unbounded.  An increment
    at or below the unit roundoff of the arithmetic relative to ||x_c|| is rounding noise: its ratio
    to the previous one says nothing about the error, and the estimate is the increment itself.
    ``history`` holds the increment norms of the earlier cycles and is extended with this one.
    Relative to ||x_c||.
    """
    norms = history + [ynorm]
    history.append(ynorm)
    rel = ynorm / xnorm if xnorm > 0 else 0.0
    if rel <= unit_roundoff:
        return rel
    if len(norms) < 2:
        return np.inf
    q = 0.0
    for i in range(max(1, len(norms) - TAIL_RATIOS), len(norms)):
        prev, cur = norms[i - 1], norms[i]
        q = max(q, cur / prev if prev > 0 else (np.inf if cur > 0 else 0.0))
    return rel * q / (1.0 - q) if q < 1.0 else np.inf


TAIL_RATIOS = 3  # contraction ratios the stopping estimate takes the largest of


# ----------------------------------------------------------------------------- driver
@dataclass
class SolveInfo:
    status: str = "ok"
    cycles: int = 0
    matvecs: int = 0
    est_rel_update: float = np.inf
    err_est: float = np.inf  # tail_estimate of the last cycle (the stopping test)
    quad_rule_error: float = 0.0
    kappa_T: float = 1.0     # max over cycles of max_i T_ii / min_i T_ii (a lower bound on cond_2(S W))
    history: list = field(default_factory=list)


def restart_solve(A, b, fun, t: float = 1.0, m: int = 20, k: int | None = None, S=None,
                  tol: float = 1e-10, max_cycles: int = 100, method: str = "sketched",
                  evaluation: str = "quadrature", n_quad: int | None = None, spec=None,
                  orth: str = "sketch", keep_cycles: bool = False):
    """Restarted Krylov approximation of f(A) b (Alg. 2 with the cycle and restart above).

    method="sketched": window-truncated randomized Arnoldi + whitening (needs S, k);
    method="plain":    classical restarted Arnoldi with CGS2 (the paper's restart).
    evaluation="quadrature" (fixed m x m work per cycle) or "growing" (dense f(M_c)).
    Returns (x, SolveInfo).
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    info = SolveInfo()
    if evaluation == "growing":
        ev = GrowingRestart(fun, t)
    else:
        rule = make_rule(fun, t, n_quad, spec)
        ev = QuadratureRestart(*rule)
        info.quad_rule_error = quadrature.rule_error(fun, *rule, t=t, spec=spec)
    v = b
    ynorms = []
    for c in range(max_cycles):
        if method == "sketched":
            cyc = sketched_cycle(A, S, v, m, k if k is not None else m, orth)
        elif method == "plain":
            cyc = arnoldi_cycle(A, v, m)
        else:
            raise ValueError(method)
        g = ev.step(cyc.X, cyc.h, cyc.beta)
        y = cyc.basis_apply(g)
        x = x + y
        info.cycles = c + 1
        info.matvecs += cyc.m
        dT = np.diag(cyc.T)
        info.kappa_T = max(info.kappa_T, float(dT.max() / dT.min()))
        nx, ny = np.linalg.norm(x), np.linalg.norm(y)
        info.est_rel_update = ny / nx if nx > 0 else 0.0
        info.err_est = tail_estimate(ny, nx, ynorms)
        rec = {"X": cyc.X, "h": cyc.h, "beta": cyc.beta, "alpha": cyc.alpha, "T": cyc.T,
               "g": g, "est": info.est_rel_update, "err_est": info.err_est, "m": cyc.m}
        if keep_cycles:
            rec["cycle"] = cyc
        info.history.append(rec)
        if cyc.breakdown:
            info.status = "breakdown"
            break
        if info.err_est <= tol:
            info.status = "ok"
            break
        v = cyc.vhat
    else:
        info.status = "not_converged"
    return x, info
