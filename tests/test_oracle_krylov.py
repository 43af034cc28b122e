"""Pins for the Krylov twins: reductions, exactness results and identities of the paper."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import workloads as wl
from oracle import exact, krylov, quadrature, sketch


def _rand_nonsym(n, seed):
    rng = np.random.default_rng(seed)
    A = sp.random(n, n, density=0.08, random_state=seed, format="csr") + sp.diags(rng.uniform(1, 3, n))
    return sp.csr_matrix(A)


def test_polynomial_exactness_one_cycle():
    """Proposition (eq. rand_arnoldi_polynomial): f of degree < m is reproduced exactly, any S and k."""
    A = _rand_nonsym(300, 0)
    b = wl.gaussian_vector(300, 1)
    S = sketch.sketch_matrix(300, 24, 4, seed=5)
    sq = lambda M: M @ M
    x, info = krylov.restart_solve(A, b, sq, m=6, k=2, S=S, max_cycles=1, evaluation="growing")
    ref = A @ (A @ b)
    assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(ref)


def test_full_dimension_is_exact():
    """m >= dim K(A, b) gives f(A) b exactly (here via a breakdown at the dimension)."""
    A = wl.laplacian_2d(5)
    As = A.to_scipy()
    b = wl.gaussian_vector(25, 2)
    S = sketch.sketch_matrix(25, 26, 25, seed=1)
    x, info = krylov.restart_solve(As, b, "exp", t=0.01, m=25, k=2, S=S, tol=1e-14, evaluation="growing")
    ref = sla.expm(-0.01 * As.toarray()) @ b
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)


def test_window_at_least_m_gives_identity_whitening():
    """k >= m: RGS keeps S W orthonormal, so T = I, X = R_m and h = r_{m+1,m} (restart-rand)."""
    A = wl.convdiff_3d(8, 20.0).to_scipy()
    b = wl.gaussian_vector(A.shape[0], 3)
    S = sketch.sketch_matrix(A.shape[0], 120, 8, seed=4)
    c = krylov.sketched_cycle(A, S, b, m=20, k=20)
    assert np.linalg.norm(c.T - np.eye(21)) < 1e-12
    assert np.linalg.norm(c.X - c.R[:20, :20]) < 1e-12 * np.linalg.norm(c.R)
    assert abs(c.h - c.R[20, 19]) < 1e-12 * abs(c.h)


def test_identity_sketch_reduces_to_arnoldi():
    """S = I_n with k >= m: randomized Arnoldi is classical (MGS) Arnoldi."""
    A = _rand_nonsym(60, 4)
    b = wl.gaussian_vector(60, 5)
    S = sp.identity(60, format="csr")
    c1 = krylov.sketched_cycle(A, S, b, m=12, k=12)
    c2 = krylov.arnoldi_cycle(A, b, m=12)
    assert np.allclose(c1.W[:, :13], c2.W[:, :13], atol=1e-12)
    assert np.allclose(c1.X, c2.X, atol=1e-11)
    assert abs(c1.h - c2.h) < 1e-11


def test_similarity_lemma():
    """Lemma (eq. similarity): Z R Z^-1 = H - (r/z_mm) c e_m^T with W = V Z, c = V^T w_{m+1}."""
    A = _rand_nonsym(80, 6)
    b = wl.gaussian_vector(80, 7)
    S = sketch.sketch_matrix(80, 40, 8, seed=8)
    W, U, R, alpha, m_eff, brk = krylov.randomized_arnoldi_window(A, S, b, 8, 8)
    m = 8
    V, Z = np.linalg.qr(W[:, :m])
    s = np.sign(np.diag(Z))
    V, Z = V * s, Z * s[:, None]
    H = V.T @ (A @ V)
    c = V.T @ W[:, m]
    lhs = Z @ R[:m, :m] @ np.linalg.inv(Z)
    rhs = H - (R[m, m - 1] / Z[m - 1, m - 1]) * np.outer(c, np.eye(m)[m - 1])
    assert np.linalg.norm(lhs - rhs) < 1e-10 * np.linalg.norm(H)


def test_whitened_arnoldi_relation():
    """A V = V X + h v_hat e_m^T and S v_hat has unit norm after whitening (truncated k)."""
    A = wl.convdiff_3d(10, 50.0).to_scipy()
    b = wl.gaussian_vector(A.shape[0], 9)
    S = sketch.sketch_matrix(A.shape[0], 80, 8, seed=1)
    c = krylov.sketched_cycle(A, S, b, m=20, k=2)
    V = c.W[:, :20] @ c.Tinv
    res = A @ V - V @ c.X - c.h * np.outer(c.vhat, np.eye(20)[19])
    assert np.linalg.norm(res) < 1e-10 * np.linalg.norm(A @ V)
    assert abs(np.linalg.norm(S @ c.vhat) - 1.0) < 1e-10
    assert np.linalg.norm(b - c.beta * V[:, 0]) < 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("fun,t", [("exp", 2e-3), ("invsqrt", 1.0), ("phi1", 2e-3), ("cos_sqrt", 0.1)])
def test_quadrature_restart_equals_growing_matrix(fun, t):
    """The quadrature recursion reproduces block c of f(M_c) e_1 over many cycles."""
    if fun in ("exp", "phi1"):
        A = wl.convdiff_3d(12, 20.0).to_scipy()
        spec = None
    else:
        A = wl.shifted_laplacian_3d(12, 1.0).to_scipy()
        spec = (3 * np.pi ** 2 + 1, 12 * 13 ** 2 + 1)
    b = wl.gaussian_vector(A.shape[0], 10)
    S = sketch.sketch_matrix(A.shape[0], 40, 8, seed=2)
    kw = dict(m=8, k=2, S=S, tol=0.0, max_cycles=6, spec=spec)
    xq, iq = krylov.restart_solve(A, b, fun, t, evaluation="quadrature", **kw)
    xg, ig = krylov.restart_solve(A, b, fun, t, evaluation="growing", **kw)
    for hq, hg in zip(iq.history, ig.history):
        assert np.linalg.norm(hq["g"] - hg["g"]) <= 1e-11 * np.linalg.norm(xg) + 1e-300
    assert np.linalg.norm(xq - xg) <= 1e-11 * np.linalg.norm(xg)


def test_scaling_invariance():
    A = wl.laplacian_2d(20).to_scipy()
    b = wl.gaussian_vector(400, 11)
    S = sketch.sketch_matrix(400, 40, 8, seed=3)
    x1, _ = krylov.restart_solve(A, b, "exp", 1e-3, m=10, k=2, S=S, tol=1e-12)
    x3, _ = krylov.restart_solve(A, 3.0 * b, "exp", 1e-3, m=10, k=2, S=S, tol=1e-12)
    assert np.linalg.norm(x3 - 3.0 * x1) <= 1e-13 * np.linalg.norm(x3)


def test_breakdown_on_eigenvector_is_exact():
    N = 16
    Phi, lam = exact.sine_basis(N)
    v = np.kron(Phi[:, 2], Phi[:, 4])                 # eigenvector of the 2-D Laplacian
    A = wl.laplacian_2d(N).to_scipy()
    S = sketch.sketch_matrix(N * N, 40, 8, seed=1)
    x, info = krylov.restart_solve(A, v, "exp", 1e-3, m=10, k=2, S=S, tol=1e-12)
    assert info.status == "breakdown" and info.cycles == 1
    ref = np.exp(-1e-3 * (lam[2] + lam[4])) * v
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)


def test_laplacian_2d_64_closed_form():
    """The 4096-row workload: tol 1e-10, relative error against the sine closed form."""
    A = wl.laplacian_2d(64)
    b = wl.gaussian_vector(A.n, 0)
    S = sketch.sketch_matrix(A.n, 80, 8, seed=1)
    ref = exact.sine_fab("exp", b, 64, [1, 1], t=1e-3)
    x, info = krylov.restart_solve(A.to_scipy(), b, "exp", 1e-3, m=20, k=2, S=S, tol=1e-10)
    assert info.status == "ok"
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)
    assert info.quad_rule_error < 1e-11


@pytest.mark.parametrize("method", ["sketched", "plain"])
def test_convdiff_small_vs_kronecker(method):
    N = 24
    A = wl.convdiff_3d(N, 50.0)
    b = wl.gaussian_vector(A.n, 0)
    t = 20.0 / (12 * (N + 1) ** 2)
    factors, _ = exact.problem_factors("convdiff_3d", N, peclet=50.0)
    ref = exact.kron_exp_fab(b, factors, t)
    S = sketch.sketch_matrix(A.n, 200, 8, seed=1)
    x, info = krylov.restart_solve(A.to_scipy(), b, "exp", t, m=50, k=4, S=S, tol=1e-8, method=method)
    assert np.linalg.norm(x - ref) <= 1e-8 * np.linalg.norm(ref)


def test_invsqrt_shifted_laplacian_closed_form():
    N = 16
    A = wl.shifted_laplacian_3d(N, 1.0)
    b = wl.gaussian_vector(A.n, 0)
    ref = exact.sine_fab("invsqrt", b, N, [1, 1, 1], 1.0)
    spec = (3 * 4 * (N + 1) ** 2 * np.sin(np.pi / (2 * (N + 1))) ** 2 + 1, 12 * (N + 1) ** 2 + 1)
    S = sketch.sketch_matrix(A.n, 120, 8, seed=1)
    x, info = krylov.restart_solve(A.to_scipy(), b, "invsqrt", m=30, k=2, S=S, tol=1e-10,
                                   spec=spec, max_cycles=200)
    assert info.status == "ok", info.cycles
    assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)


def test_unrestarted_arnoldi_matches_closed_form():
    A = wl.laplacian_2d(30)
    b = wl.gaussian_vector(A.n, 4)
    ref = exact.sine_fab("exp", b, 30, [1, 1], t=1e-3)
    x = krylov.arnoldi_full(A.to_scipy(), b, 60, "exp", 1e-3)
    assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(ref)


def test_fixed_rules_converge_to_the_same_result_at_high_condition_number():
    """z^(-1/2) of a 3-D Laplacian shifted to condition number 2.6e4 (Section 4's quadrature-based
    restart with the tan-substituted Stieltjes rule): increments grow transiently over the cycles,
    yet the fixed rule r converges to r(A) b and the result meets the closed form; the main and check
    rules agree on every cycle's projected matrix."""
    N = 16
    lmin0 = 3 * 4 * (N + 1) ** 2 * np.sin(np.pi / (2 * (N + 1))) ** 2
    lmax = 12 * (N + 1) ** 2
    shift = lmax / 2.6e4 - lmin0
    A = wl.shifted_laplacian_3d(N, shift)
    b = wl.gaussian_vector(A.n, 0)
    spec = (lmin0 + shift, lmax + shift)
    S = sketch.sketch_matrix(A.n, 120, 8, seed=1)
    x, info = krylov.restart_solve(A.to_scipy(), b, "invsqrt", m=30, k=2, S=S, tol=1e-10, max_cycles=400,
                                   spec=spec)
    ref = exact.sine_fab("invsqrt", b, N, [1, 1, 1], shift)
    assert info.status == "ok" and info.cycles > 50
    assert np.linalg.norm(x - ref) <= 1e-8 * np.linalg.norm(ref)
    assert info.quad_rule_error <= 1e-11


def test_fixed_rule_iteration_converges_to_r_of_A():
    """With a deliberately coarse rule r (6 nodes for z^(-1/2)), the restarted iteration converges
    to r(A) b, not to f(A) b: x matches r(A) b from the eigendecomposition, and the gap to f(A) b
    stays within the sampled rule error (the quantity the solver reports)."""
    N = 10
    A = wl.shifted_laplacian_3d(N, 1.0)
    b = wl.gaussian_vector(A.n, 4)
    lo = 3 * 4 * (N + 1) ** 2 * np.sin(np.pi / (2 * (N + 1))) ** 2 + 1.0
    hi = 12 * (N + 1) ** 2 + 1.0
    S = sketch.sketch_matrix(A.n, 60, 4, seed=2)
    x, info = krylov.restart_solve(A.to_scipy(), b, "invsqrt", m=20, k=3, S=S, tol=1e-14, max_cycles=200,
                                   n_quad=6, spec=(lo, hi))
    lam, Q = np.linalg.eigh(A.to_scipy().toarray())
    zeta, w, _ = krylov.make_rule("invsqrt", n_quad=6, spec=(lo, hi))
    r = quadrature.rational_scalar(zeta, w, lam).real
    rA_b = Q @ (r * (Q.T @ b))
    fA_b = Q @ ((Q.T @ b) / np.sqrt(lam))
    assert np.linalg.norm(x - rA_b) <= 1e-11 * np.linalg.norm(rA_b)
    gap = np.linalg.norm(rA_b - fA_b) / np.linalg.norm(fA_b)
    assert 1e-8 < gap <= info.quad_rule_error


def test_kappa_T_is_a_lower_bound_on_the_basis_condition():
    """kappa_T (the spread of T's positive diagonal, max over cycles) is >= 1 and <= cond_2(S W) of
    every cycle (a triangular matrix's condition number is at least its diagonal spread); the plain
    method's T is the identity."""
    A = wl.convdiff_3d(12, 20.0)
    b = wl.gaussian_vector(A.n, 3)
    S = sketch.sketch_matrix(A.n, 60, 4, seed=2)
    x, info = krylov.restart_solve(A.to_scipy(), b, "exp", 2e-3, m=20, k=2, S=S, tol=1e-12, max_cycles=6,
                                   keep_cycles=True)
    ratios = []
    for rec in info.history:
        cyc = rec["cycle"]
        cols = cyc.m if cyc.breakdown else cyc.m + 1
        dT = np.diag(cyc.T)
        ratios.append(dT.max() / dT.min())
        assert dT.max() / dT.min() <= np.linalg.cond(cyc.U[:, :cols]) * (1 + 1e-10)
    assert info.kappa_T == pytest.approx(max(ratios), rel=0, abs=0)
    assert info.kappa_T >= 1.0 and len(ratios) >= 2
    _, plain = krylov.restart_solve(A.to_scipy(), b, "exp", 2e-3, m=20, method="plain", tol=1e-12, max_cycles=3)
    assert plain.kappa_T == 1.0


def test_full_space_window_with_k_at_least_m_is_classical_arnoldi():
    """O2d (full-space inner products) with k >= m is modified Gram-Schmidt Arnoldi, which spans the
    same Krylov basis as the CGS2 Arnoldi twin: W equals V and R equals H (Section 2.2)."""
    A = _rand_nonsym(90, 12)
    b = wl.gaussian_vector(90, 13)
    S = sketch.sketch_matrix(90, 40, 8, seed=3)
    W, U, R, alpha, m_eff, brk = krylov.randomized_arnoldi_window(A, S, b, 12, 12, orth="full")
    c = krylov.arnoldi_cycle(A, b, m=12)
    assert not brk and m_eff == 12
    assert abs(alpha - np.linalg.norm(b)) <= 1e-14 * np.linalg.norm(b)
    assert np.allclose(W, c.W, atol=1e-12)
    assert np.allclose(R, c.R, atol=1e-11 * np.abs(c.R).max())
    assert np.allclose(U, S @ W, atol=1e-13)


def test_full_space_window_is_incomplete_orthogonalization():
    """O2d with k < m: A W_m = W_{m+1} R with R upper Hessenberg and banded (entries i >= j - k + 1
    only), every w_j of unit 2-norm and orthogonal to the k vectors before it (incomplete
    orthogonalization, Section 3), while vectors further back are not orthogonal."""
    A = wl.convdiff_3d(9, 40.0).to_scipy()
    n = A.shape[0]
    b = wl.gaussian_vector(n, 14)
    S = sketch.sketch_matrix(n, 60, 8, seed=5)
    m, k = 16, 3
    W, U, R, alpha, m_eff, brk = krylov.randomized_arnoldi_window(A, S, b, m, k, orth="full")
    assert not brk
    assert np.linalg.norm(A @ W[:, :m] - W @ R) <= 1e-12 * np.linalg.norm(A @ W[:, :m])
    i, j = np.indices(R.shape)
    assert np.all(R[(i < j - k + 1) | (i > j + 1)] == 0.0)
    assert np.allclose(np.linalg.norm(W, axis=0), 1.0, atol=1e-13)
    G = W.T @ W
    for jj in range(1, m + 1):
        for ii in range(max(0, jj - k), jj):
            assert abs(G[ii, jj]) <= 1e-12
    assert np.max(np.abs(np.triu(G, k + 1))) > 1e-6
    assert np.allclose(U, S @ W, atol=1e-13)


@pytest.mark.parametrize("k", [2, 16])
def test_identity_sketch_makes_both_inner_products_equal(k):
    """With S = I_n the sketched and the full-space inner products coincide, so the two
    orthogonalizations of O2 produce the same window-truncated basis for any k."""
    A = _rand_nonsym(70, 15)
    b = wl.gaussian_vector(70, 16)
    S = sp.identity(70, format="csr")
    r1 = krylov.randomized_arnoldi_window(A, S, b, 16, k, orth="sketch")
    r2 = krylov.randomized_arnoldi_window(A, S, b, 16, k, orth="full")
    assert np.allclose(r1[0], r2[0], atol=1e-12)
    assert np.allclose(r1[2], r2[2], atol=1e-11 * np.abs(r2[2]).max())
    assert r1[4:] == r2[4:]


def test_full_space_window_solve_meets_the_closed_form():
    """The O2d restarted solve (full-space truncated orthogonalization, whitened by the sketch)
    converges to the same f(A) b as the sketched method on the 2-D Laplacian."""
    A = wl.laplacian_2d(24)
    b = wl.gaussian_vector(A.n, 17)
    S = sketch.sketch_matrix(A.n, 80, 8, seed=1)
    ref = exact.sine_fab("exp", b, 24, [1, 1], t=1e-3)
    x, info = krylov.restart_solve(A.to_scipy(), b, "exp", 1e-3, m=20, k=2, S=S, tol=1e-11, orth="full")
    assert info.status == "ok"
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)


# ------------------------------------------------------------------- stopping test (tail estimate)
def test_tail_estimate_is_exact_for_geometric_increments():
    """Increments y_c = q^(c-1) v add up to x* = v / (1 - q); after cycle c the remaining error is
    q^c ||v|| / (1 - q), which the tail estimate returns exactly (relative to ||x_c||) from the
    second cycle on; after the first cycle there is no ratio and the estimate is unbounded."""
    v = np.random.default_rng(3).standard_normal(40)
    for q in (0.05, 0.5, 0.93):
        hist, x = [], np.zeros_like(v)
        xstar = v / (1.0 - q)
        for c in range(1, 14):
            y = q ** (c - 1) * v
            x = x + y
            est = krylov.tail_estimate(np.linalg.norm(y), np.linalg.norm(x), hist)
            true = np.linalg.norm(xstar - x) / np.linalg.norm(x)
            if c == 1:
                assert est == np.inf
            else:
                assert est == pytest.approx(true, rel=1e-10), (q, c)


def test_tail_estimate_uses_the_largest_of_three_ratios():
    """A small ratio right after growth (a dip inside a transient) gives no bound: the estimate takes
    the largest of the last three ratios.  Hand-computed values; a zero increment gives 0."""
    hist = []
    ests = [krylov.tail_estimate(y, 1.0, hist) for y in (1.0, 0.1, 0.5, 1e-3, 5e-4, 4e-4, 2e-4)]
    assert ests[0] == np.inf                                  # no ratio yet
    assert ests[1] == pytest.approx(0.1 * 0.1 / 0.9)          # one ratio, 0.1
    assert ests[2] == np.inf                                  # ratio 5
    assert ests[3] == np.inf                                  # ratios 2e-3, 5, 0.1
    assert ests[4] == np.inf                                  # ratios 0.5, 2e-3, 5
    assert ests[5] == pytest.approx(4e-4 * 0.8 / 0.2)         # ratios 0.8, 0.5, 2e-3
    assert ests[6] == pytest.approx(2e-4 * 0.8 / 0.2)         # ratios 0.5, 0.8, 0.5
    assert krylov.tail_estimate(0.0, 1.0, [1.0, 0.5]) == 0.0


def test_tail_estimate_at_the_rounding_level():
    """Increments that have shrunk to the unit roundoff relative to ||x|| and then scatter (ratios
    above 1) end the test with the increment itself as the estimate; the same ratios above the
    roundoff keep it unbounded.  Hand-computed values, FP64 roundoff 2^-53 = 1.11e-16."""
    hist = []
    ests = [krylov.tail_estimate(y, 1.0, hist) for y in (1.0, 1e-3, 1e-9, 1e-17, 3e-17, 2e-17)]
    assert ests[0] == np.inf
    assert ests[1] == pytest.approx(1e-3 * 1e-3 / (1 - 1e-3))
    assert ests[2] == pytest.approx(1e-9 * 1e-3 / (1 - 1e-3))   # ratios 1e-6, 1e-3
    assert ests[3:] == [1e-17, 3e-17, 2e-17]                   # at the roundoff: ratios ignored
    hist = []
    ests = [krylov.tail_estimate(y, 1.0, hist) for y in (1.0, 1e-3, 1e-9, 1e-14, 3e-14)]
    assert ests[4] == np.inf                                   # ratio 3 above the roundoff
    hist = []
    assert [krylov.tail_estimate(y, 1.0, hist, unit_roundoff=2.0 ** -24) for y in (1.0, 1e-6, 5e-8)] == \
        [np.inf, pytest.approx(1e-6 * 1e-6 / (1 - 1e-6)), 5e-8]  # FP32 roundoff 5.96e-8
    assert krylov.tail_estimate(0.0, 1.0, [1.0, 0.5]) == 0.0


def test_tail_estimate_stops_within_tol_where_the_raw_difference_does_not():
    """z^(-1/2) of the 3-D Laplacian shifted to condition number 2.6e4, d = 4m: the increments of
    the restart swing by two orders of magnitude from cycle to cycle.  Stopping at the first cycle
    whose raw difference ||y_c|| / ||x_c|| is below tol leaves an error above tol (the sine closed
    form decides); the tail estimate stops later with the error within tol."""
    N, tol = 16, 1e-4
    lmin0 = 3 * 4 * (N + 1) ** 2 * np.sin(np.pi / (2 * (N + 1))) ** 2
    lmax = 12 * (N + 1) ** 2
    shift = lmax / 2.6e4 - lmin0
    A = wl.shifted_laplacian_3d(N, shift)
    b = wl.gaussian_vector(A.n, 0)
    spec = (lmin0 + shift, lmax + shift)
    S = sketch.sketch_matrix(A.n, 120, 8, seed=1)
    ref = exact.sine_fab("invsqrt", b, N, [1, 1, 1], shift)
    x, info = krylov.restart_solve(A.to_scipy(), b, "invsqrt", m=30, k=2, S=S, tol=tol, max_cycles=300,
                                   spec=spec, keep_cycles=True)
    assert info.status == "ok"
    assert np.linalg.norm(x - ref) <= tol * np.linalg.norm(ref)
    xs = np.zeros_like(b)
    for c, h in enumerate(info.history):
        xs = xs + h["cycle"].basis_apply(h["g"])
        if h["est"] <= tol:  # where the raw successive difference would have stopped
            assert c + 1 < info.cycles
            assert np.linalg.norm(xs - ref) > tol * np.linalg.norm(ref)
            break
    else:
        raise AssertionError("the raw difference never fell below tol")


@pytest.mark.parametrize("fun,t", [("phi1", 1e-3), ("phi1", 2e-2), ("cos_sqrt", 0.02), ("cos_sqrt", 0.2)])
def test_phi1_and_cos_sqrt_restarts_meet_the_closed_form(fun, t):
    """phi_1(-t A) b (eq. conv_diff_sol3) and cos(t sqrt A) b (eq. drum_sol) by the sketched restart on
    the 2-D Laplacian, N = 32, against the sine closed form."""
    N = 32
    A = wl.laplacian_2d(N)
    b = wl.gaussian_vector(A.n, 13)
    spec = (8 * (N + 1) ** 2 * np.sin(np.pi / (2 * (N + 1))) ** 2, 8 * (N + 1) ** 2)
    S = sketch.sketch_matrix(A.n, 80, 8, seed=1)
    x, info = krylov.restart_solve(A.to_scipy(), b, fun, t, m=20, k=2, S=S, tol=1e-11, max_cycles=200,
                                   spec=spec if fun == "cos_sqrt" else None)
    ref = exact.sine_fab(fun, b, N, [1, 1], 0.0, t)
    assert info.status == "ok", info.cycles
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)
    assert info.quad_rule_error <= 1e-11
