"""Pins for the exact f(A)b oracles (closed forms vs dense evaluation) and for the inputs."""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as wl
from oracle import exact


def test_sine_basis_is_eigenbasis():
    N = 17
    Phi, lam = exact.sine_basis(N)
    T = exact.laplace_factor(N)
    assert np.allclose(T @ Phi, Phi * lam[None, :], rtol=0, atol=1e-9 * lam.max())
    assert np.allclose(Phi @ Phi, np.eye(N), atol=1e-13)


@pytest.mark.parametrize("kind,N,kw,fun,t", [
    ("laplacian_2d", 11, {}, "exp", 1e-3),
    ("anisotropic_2d", 9, {"cy": 0.01}, "exp", 1e-3),
    ("shifted_laplacian_3d", 5, {"shift": 1.0}, "invsqrt", 1.0),
    ("shifted_laplacian_3d", 5, {"shift": 1.0}, "exp", 1e-2),
])
def test_sine_closed_form_vs_dense(kind, N, kw, fun, t):
    factors, shift = exact.problem_factors(kind, N, **kw)
    A = exact.assemble_dense(factors, shift)
    b = wl.gaussian_vector(A.shape[0], 0)
    coefs = {"laplacian_2d": [1, 1], "anisotropic_2d": [1, kw.get("cy")],
             "shifted_laplacian_3d": [1, 1, 1]}[kind]
    x1 = exact.sine_fab(fun, b, N, coefs, shift, t)
    x2 = (sla.expm(-t * A) if fun == "exp" else np.linalg.inv(sla.sqrtm(A)).real) @ b
    assert np.linalg.norm(x1 - x2) <= 1e-12 * np.linalg.norm(x2)


@pytest.mark.parametrize("transpose", [False, True])
def test_kron_exp_nonsymmetric_vs_dense(transpose):
    N = 6
    factors, _ = exact.problem_factors("convdiff_3d", N, peclet=20.0)
    A = exact.assemble_dense(factors)
    assert np.linalg.norm(A - A.T) > 1.0           # genuinely non-symmetric
    b = wl.gaussian_vector(N ** 3, 1)
    t = 2e-3
    x1 = exact.kron_exp_fab(b, factors, t, transpose=transpose)
    x2 = sla.expm(-t * (A.T if transpose else A)) @ b
    assert np.linalg.norm(x1 - x2) <= 1e-13 * np.linalg.norm(x2)


@pytest.mark.parametrize("build,kind,kw", [
    (lambda N: wl.laplacian_2d(N), "laplacian_2d", {}),
    (lambda N: wl.anisotropic_2d(N, 0.01), "anisotropic_2d", {"cy": 0.01}),
    (lambda N: wl.convdiff_3d(N, 50.0), "convdiff_3d", {"peclet": 50.0}),
    (lambda N: wl.shifted_laplacian_3d(N, 1.0), "shifted_laplacian_3d", {"shift": 1.0}),
])
def test_csr_inputs_equal_operator_definition(build, kind, kw):
    """The CSR generator and the oracle's own factors describe the same operator."""
    N = 5
    A = build(N)
    factors, shift = exact.problem_factors(kind, N, **kw)
    D = exact.assemble_dense(factors, shift)
    assert np.array_equal(A.to_scipy().toarray(), D) or np.allclose(A.to_scipy().toarray(), D, rtol=1e-15, atol=0)
    rp = A.rowptr
    for i in range(A.n):                                       # sorted, in-range columns
        c = A.colind[rp[i]:rp[i + 1]]
        assert np.all(np.diff(c) > 0) and c.min() >= 0 and c.max() < A.n


def test_published_sizes():
    assert (wl.laplacian_2d(64).n, wl.laplacian_2d(64).nnz) == (4096, 20224)
    A = wl.convdiff_3d(96, 20.0)
    assert (A.n, A.nnz) == (884736, 6137856)


def test_kron_sum_apply_matches_csr():
    A = wl.convdiff_3d(7, 20.0)
    factors, _ = exact.problem_factors("convdiff_3d", 7, peclet=20.0)
    x = wl.gaussian_vector(A.n, 3)
    assert np.allclose(exact.kron_sum_apply(factors, x), A.to_scipy() @ x, rtol=1e-13, atol=1e-9)


def test_exp_action_grads_against_finite_differences():
    """Gradient of L = <c, exp(-t A) b> (nonsymmetric convection-diffusion) against central
    differences: exact in b (L is linear in b), O(h^2) in t."""
    N, t = 8, 1e-3
    factors, _ = exact.problem_factors("convdiff_3d", N, peclet=20.0)
    n = N ** 3
    b, c = wl.gaussian_vector(n, 1), wl.gaussian_vector(n, 2)
    L, gb, gt = exact.exp_action_grads(factors, b, c, t)
    for seed in (5, 6):
        u = wl.unit_direction(n, seed)
        h = 1e-3
        fd = (exact.exp_action_grads(factors, b + h * u, c, t)[0] - exact.exp_action_grads(factors, b - h * u, c, t)[0]) / (2 * h)
        assert abs(fd - gb @ u) <= 1e-10 * max(abs(fd), 1.0)
    ht = 1e-4 * t
    fdt = (exact.exp_action_grads(factors, b, c, t + ht)[0] - exact.exp_action_grads(factors, b, c, t - ht)[0]) / (2 * ht)
    assert abs(fdt - gt) <= 1e-7 * abs(gt)
    # the adjoint differs from the forward operator for this nonsymmetric A
    assert np.linalg.norm(gb - exact.kron_exp_fab(c, factors, t)) > 1e-3 * np.linalg.norm(gb)


@pytest.mark.parametrize("fun,t", [("exp", 2e-3), ("invsqrt", 1.0), ("phi1", 2e-3), ("cos_sqrt", 0.05)])
def test_dense_fab_matches_sine_closed_form(fun, t):
    """O1c (dense f of the assembled matrix, for tiny operators of any structure) against the sine
    eigenbasis closed form on the 2-D Laplacian shifted by 1 (SPD, so z^(-1/2) is defined)."""
    N = 9
    factors, shift = [exact.laplace_factor(N)] * 2, 1.0
    A = exact.assemble_dense(factors, shift)
    b = wl.gaussian_vector(N * N, 3)
    x1 = exact.dense_fab(fun, A, b, t)
    x2 = exact.sine_fab(fun, b, N, [1, 1], shift, t)
    assert np.linalg.norm(x1 - x2) <= 1e-12 * np.linalg.norm(x2)


def test_dense_fab_matches_kronecker_exp_nonsymmetric():
    """O1c against the Kronecker-exp identity (O1b) on a non-symmetric convection-diffusion operator."""
    N = 5
    factors, _ = exact.problem_factors("convdiff_3d", N, peclet=30.0)
    A = exact.assemble_dense(factors)
    b = wl.gaussian_vector(N ** 3, 4)
    x1 = exact.dense_fab("exp", A, b, 3e-3)
    x2 = exact.kron_exp_fab(b, factors, 3e-3)
    assert np.linalg.norm(x1 - x2) <= 1e-13 * np.linalg.norm(x2)


@pytest.mark.parametrize("N,t", [(7, 1e-3), (9, 3e-2)])
def test_phi1_and_cos_sqrt_closed_forms_vs_scipy(N, t):
    """The sine closed forms of phi_1(-t A) b and cos(t sqrt A) b against scipy's dense routes on the
    assembled 2-D Laplacian (SPD): (t A)^(-1) (I - e^(-t A)) b and cosm(t sqrtm(A)) b."""
    factors, shift = exact.problem_factors("laplacian_2d", N)
    A = exact.assemble_dense(factors, shift)
    b = wl.gaussian_vector(N * N, 11)
    x1 = exact.sine_fab("phi1", b, N, [1, 1], 0.0, t)
    x2 = np.linalg.solve(t * A, b - sla.expm(-t * A) @ b)
    assert np.linalg.norm(x1 - x2) <= 1e-12 * np.linalg.norm(x2)
    tc = 3.0 / np.sqrt(8 * (N + 1) ** 2)
    y1 = exact.sine_fab("cos_sqrt", b, N, [1, 1], 0.0, tc)
    y2 = sla.cosm(tc * sla.sqrtm(A).real) @ b
    assert np.linalg.norm(y1 - y2) <= 1e-11 * np.linalg.norm(y2)


def test_phi1_dense_nonsymmetric_vs_scipy():
    """O1c's phi_1 (augmented exponential) on a non-symmetric convection-diffusion operator against
    (t A)^(-1) (I - e^(-t A)) b with scipy's expm."""
    N, t = 5, 4e-3
    factors, _ = exact.problem_factors("convdiff_3d", N, peclet=30.0)
    A = exact.assemble_dense(factors)
    b = wl.gaussian_vector(N ** 3, 12)
    x1 = exact.dense_fab("phi1", A, b, t)
    x2 = np.linalg.solve(t * A, b - sla.expm(-t * A) @ b)
    assert np.linalg.norm(x1 - x2) <= 1e-12 * np.linalg.norm(x2)
