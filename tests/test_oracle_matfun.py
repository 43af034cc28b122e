"""Pins for the dense matrix functions and the quadrature rules of the oracle."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import matfun, quadrature


@pytest.mark.parametrize("theta", [0.3, 2.0, 50.0])
def test_expm_rotation_closed_form(theta):
    G = np.array([[0.0, -theta], [theta, 0.0]])
    E = matfun.expm(G)
    R = np.array([[np.cos(theta), -np.sin(theta)], [np.sin(theta), np.cos(theta)]])
    assert np.max(np.abs(E - R)) < 1e-13 * max(1.0, theta)


def test_expm_nilpotent_and_diagonal():
    N = np.triu(np.random.default_rng(0).standard_normal((4, 4)), 1)
    assert np.allclose(matfun.expm(N), np.eye(4) + N + N @ N / 2 + N @ N @ N / 6, atol=1e-14, rtol=0)
    d = np.array([-30.0, -1.0, 0.5, 3.0])
    assert np.allclose(matfun.expm(np.diag(d)), np.diag(np.exp(d)), rtol=1e-14, atol=0)


def test_pade13_accuracy_at_threshold():
    """The [13/13] approximant meets unit roundoff at |x| = theta_13 (the scaling threshold)."""
    c = matfun.PADE13
    for x in (matfun.THETA13, -matfun.THETA13, 1.0):
        num = np.polyval(c[::-1], x)
        den = np.polyval(c[::-1], -x)
        assert abs(num / den / np.exp(x) - 1.0) < 2e-15


def test_expm_matches_scipy_nonnormal():
    rng = np.random.default_rng(1)
    for scale in (0.1, 3.0, 40.0):
        A = scale * rng.standard_normal((12, 12)) / 4
        A += np.triu(rng.standard_normal((12, 12)), 1) * scale
        E1, E2 = matfun.expm(A), sla.expm(A)
        assert np.linalg.norm(E1 - E2) <= 1e-12 * np.linalg.norm(E2) * max(1, scale)


def test_invsqrt_closed_form_and_identity():
    rng = np.random.default_rng(2)
    Q, _ = np.linalg.qr(rng.standard_normal((8, 8)))
    lam = np.geomspace(0.5, 300.0, 8)
    A = Q @ np.diag(lam) @ Q.T
    Y = matfun.invsqrt(A)
    assert np.allclose(Y, Q @ np.diag(lam ** -0.5) @ Q.T, rtol=0, atol=1e-12)
    B = A + np.triu(rng.standard_normal((8, 8)), 1)        # non-normal, same spectrum
    Yb = matfun.invsqrt(B)
    assert np.linalg.norm(Yb @ Yb @ B - np.eye(8)) < 1e-10


def _sector_points(n=400):
    """Points s = -t z with Re s in [-45, 0.5] and |Im s| <= 0.75 |Re s| + 4 (sketched Ritz region)."""
    rng = np.random.default_rng(3)
    re = rng.uniform(-45.0, 0.5, n)
    im = rng.uniform(-1, 1, n) * (0.75 * np.abs(re) + 4.0)
    return re + 1j * im


@pytest.mark.parametrize("t", [1e-3, 1e-4, 1.0])
def test_exp_rule_scalar_accuracy(t):
    s = _sector_points()
    z = -s / t
    P, mu, L = quadrature.EXP_MAIN[1:]
    for N in (quadrature.EXP_MAIN[0], 160):
        zeta, w = quadrature.exp_rule(t, N, P, mu, L)
        r = quadrature.rational_scalar(zeta, w, z)
        err = np.abs(r - np.exp(-t * z))
        assert err.max() < 1e-12, (N, err.max())


def test_exp_rule_conjugate_pairs():
    zeta, w = quadrature.exp_rule(1e-3)
    zh, wh = quadrature.conjugate_half(zeta, w)
    assert len(zh) == len(zeta) // 2
    z = np.array([50.0, 2000.0, 33000.0])
    full = quadrature.rational_scalar(zeta, w, z)
    half = 2 * quadrature.rational_scalar(zh, wh, z).real
    assert np.allclose(full.real, half, rtol=1e-13, atol=1e-16)
    assert np.max(np.abs(full.imag)) < 1e-13


def test_invsqrt_rule_accuracy():
    lo, hi = 30.6, 7.93e5
    zeta, w = quadrature.invsqrt_rule(128, lo, hi)
    z = np.geomspace(lo, hi, 300)
    for zz in (z, z * np.exp(0.5j)):
        r = quadrature.rational_scalar(zeta, w, zz)
        assert np.max(np.abs(r * np.sqrt(zz) - 1.0)) < 1e-14


@pytest.mark.parametrize("fun,N,lo", [("exp", 128, None), ("exp", 24, None), ("invsqrt", 128, 0.5),
                                       ("invsqrt", 12, 0.5)])
def test_rule_error_tracks_node_count(fun, N, lo):
    """rule_error is tiny for the default rules and large for coarse ones (the quantity the solver
    compares with the tolerance)."""
    if fun == "exp":
        z, w = quadrature.conjugate_half(*quadrature.exp_rule(1e-3, N))
        e = quadrature.rule_error("exp", z, w, True, t=1e-3)
    else:
        z, w = quadrature.invsqrt_rule(N, lo, 2e4)
        e = quadrature.rule_error("invsqrt", z, w, False, spec=(lo, 2e4))
    if N >= 128:
        assert e < 1e-12
    else:
        assert e > 1e-6


# --------------------------------------------------------- phi_1 (eq. conv_diff_sol3), cos(t sqrt)
def test_phi1_closed_forms():
    """phi_1 through the augmented exponential against its definition: (e^d - 1)/d on a diagonal,
    the series I + N/2 + N^2/6 on a nilpotent N (N^3 = 0), and M phi_1(M) = e^M - I on a
    non-normal M (scipy's expm on the right-hand side)."""
    d = np.array([-40.0, -1.0, -1e-9, 0.0, 0.7, 3.0])
    ph = np.diag(matfun.phi1(np.diag(d)))
    ref = np.array([np.expm1(x) / x if x != 0 else 1.0 for x in d])
    assert np.allclose(ph, ref, rtol=1e-14, atol=0)
    N = np.triu(np.random.default_rng(5).standard_normal((3, 3)), 1)
    assert np.allclose(matfun.phi1(N), np.eye(3) + N / 2 + N @ N / 6, atol=1e-14, rtol=0)
    rng = np.random.default_rng(6)
    M = rng.standard_normal((10, 10)) + np.triu(rng.standard_normal((10, 10)), 1) * 3 - 4 * np.eye(10)
    assert np.linalg.norm(M @ matfun.phi1(M) - (sla.expm(M) - np.eye(10))) <= 1e-12 * np.linalg.norm(sla.expm(M))


def test_cos_sqrt_closed_forms():
    """cos(t sqrt A) through the first-order form: cos(t sqrt d) on a diagonal (cosh for d < 0), the
    series I - t^2 A/2 + t^4 A^2/24 on a nilpotent A (A^3 = 0), the double-angle identity
    C(2t) = 2 C(t)^2 - I on a non-normal A, and V cos(t sqrt L) V^T for a symmetric one."""
    t = 0.7
    d = np.array([-4.0, 0.0, 0.5, 9.0, 400.0])
    c = np.diag(matfun.cos_sqrt(np.diag(d), t))
    ref = np.array([np.cosh(t * np.sqrt(-x)) if x < 0 else np.cos(t * np.sqrt(x)) for x in d])
    assert np.allclose(c, ref, rtol=0, atol=1e-13)
    A = np.triu(np.random.default_rng(7).standard_normal((3, 3)), 1)
    assert np.allclose(matfun.cos_sqrt(A, t), np.eye(3) - t ** 2 * A / 2 + t ** 4 * A @ A / 24, atol=1e-14, rtol=0)
    rng = np.random.default_rng(8)
    B = rng.standard_normal((8, 8)) + 5 * np.eye(8)
    C1, C2 = matfun.cos_sqrt(B, t), matfun.cos_sqrt(B, 2 * t)
    assert np.linalg.norm(C2 - (2 * C1 @ C1 - np.eye(8))) <= 1e-12 * max(1.0, np.linalg.norm(C2))
    S = rng.standard_normal((8, 8))
    S = S @ S.T + np.eye(8)
    lam, V = np.linalg.eigh(S)
    assert np.linalg.norm(matfun.cos_sqrt(S, t) - (V * np.cos(t * np.sqrt(lam))) @ V.T) <= 1e-12 * np.sqrt(8)


@pytest.mark.parametrize("t", [1e-3, 1.0])
def test_phi1_rule_scalar_accuracy(t):
    """The Hankel contour with weights over s reproduces phi_1(-t z) on the region the exp rule
    covers (sketched Ritz values included), and its conjugate half doubles to the full rule."""
    s = _sector_points()
    z = -s / t
    zeta, w = quadrature.phi1_rule(t)
    r = quadrature.rational_scalar(zeta, w, z)
    ref = np.expm1(s) / s
    assert np.max(np.abs(r - ref)) < 1e-12
    zh, wh = quadrature.conjugate_half(zeta, w)
    x = np.array([0.0, 30.0 / t, 3e3 / t])
    assert np.allclose(2 * quadrature.rational_scalar(zh, wh, x).real, quadrature.rational_scalar(zeta, w, x).real,
                       rtol=1e-13, atol=1e-16)
    assert quadrature.rule_error("phi1", zh, wh, True, t=t) < 1e-12


@pytest.mark.parametrize("kappa", [0.3, 4.0, 20.0, 45.0, 100.0])
def test_cos_sqrt_ellipse_widens_while_the_growth_allows(kappa):
    """The ellipse parameter: rho = 2 for few oscillations, rho_min = exp(37/N) for many, and in
    between the largest candidate whose max |f| on the nodes stays within the bound.  Inside the
    chosen ellipse the rule reproduces cos(t sqrt z) directly (no quadrature), also for points
    outside [lo, hi] where sketched Ritz values can fall: out to ellipse coordinate
    |w| = rho e^(-40/N) the truncation term (|w|/rho)^N is below e^-40."""
    lo, hi, N = 30.6, 2029.0, quadrature.COS_SQRT_N
    t = kappa / np.sqrt(hi)
    rho = quadrature.cos_sqrt_rho(t, N, lo, hi)
    rho_min = np.exp(37.0 / N)
    assert rho_min - 1e-15 <= rho <= 2.0 + 1e-15
    if kappa <= 4.0:
        assert rho == pytest.approx(2.0, rel=1e-14)
    if kappa >= 100.0:
        assert rho == pytest.approx(rho_min, rel=1e-14)
    zeta, w = quadrature.cos_sqrt_rule(t, N, lo, hi)
    c, h = 0.5 * (lo + hi), 0.5 * (hi - lo)
    growth = t * np.max(np.abs(np.sqrt(zeta).imag))  # ln max |f| on the nodes, within ~ln 100 here
    assert growth <= np.log(100.0) + 1e-12 or rho == pytest.approx(rho_min, rel=1e-14)
    # points on the ellipse of radius rho e^(-40/N): the interval's ends pushed out, and off the axis
    r_in = rho * np.exp(-40.0 / N)
    ph = np.linspace(0.0, 2 * np.pi, 64, endpoint=False)
    zz = c + h * (r_in * np.exp(1j * ph) + np.exp(-1j * ph) / r_in) / 2
    r = quadrature.rational_scalar(zeta, w, zz)
    fmax = np.exp(growth)
    assert np.max(np.abs(r - np.cos(t * np.sqrt(zz)))) < 1e-12 * fmax


@pytest.mark.parametrize("kappa", [1.0, 20.0, 60.0])
def test_cos_sqrt_rule_accuracy(kappa):
    """The ellipse rule reproduces cos(t sqrt z) on [lo, hi] (t sqrt(hi) = kappa oscillations), on a
    neighbourhood of the interval inside the ellipse, and a coarse rule is flagged by rule_error."""
    lo, hi = 20.0, 3.4e4
    t = kappa / np.sqrt(hi)
    zeta, w = quadrature.cos_sqrt_rule(t, quadrature.COS_SQRT_N, lo, hi)
    x = np.linspace(lo, hi, 500)
    for zz in (x, x + 1j * 0.01 * (hi - lo) * np.sin(np.linspace(0, np.pi, 500))):
        r = quadrature.rational_scalar(zeta, w, zz)
        assert np.max(np.abs(r - np.cos(t * np.sqrt(zz)))) < 1e-11
    zh, wh = quadrature.conjugate_half(zeta, w)
    assert len(zh) == len(zeta) // 2
    assert quadrature.rule_error("cos_sqrt", zh, wh, True, t=t, spec=(lo, hi)) < 1e-11
    zc, wc = quadrature.conjugate_half(*quadrature.cos_sqrt_rule(max(t, 60 / np.sqrt(hi)), 24, lo, hi))
    assert quadrature.rule_error("cos_sqrt", zc, wc, True, t=max(t, 60 / np.sqrt(hi)), spec=(lo, hi)) > 1e-6
