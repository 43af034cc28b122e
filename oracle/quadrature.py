"""Partial-fraction quadrature rules  r(z) = sum_l w_l / (zeta_l - z)  ~  f(z).

The restart of the method keeps the projected matrix at m x m by evaluating f
through an integral representation (Section 4 names quadrature-based restarts
as the alternative to the growing f(R_km); the Cauchy integral is eq.
cauchy_def).  Discretising the integral gives a rational function in partial
fractions; the restart then evaluates r on the growing block matrix *exactly*
by block forward substitution (see ``krylov.QuadratureRestart``).

exp(-t z)  -- Cauchy integral on a parabolic Hankel contour in s = -t z:
    s(u) = P - mu u^2 + 2 i mu u,  u in [-U, U],  U = sqrt((P + L)/mu),
    N midpoint nodes u_k = -U + (k + 1/2) h, h = 2U/N.
    exp(-t X) = (1/2 pi i) int e^s (s I + t X)^{-1} ds, and
    (s I + t X)^{-1} = -(1/t) (zeta I - X)^{-1} with zeta = -s/t, so
    zeta_k = -s(u_k)/t,  w_k = -h s'(u_k) e^{s(u_k)} / (2 pi i t).
    The contour crosses the real axis at s = P and is cut where Re s = -L
    (e^-L negligible); it encloses every point s with
    Re s < P - (Im s)^2 / (4 mu).  Defaults (N, P, mu, L) = (128, 3, 6, 45).
    Design reading (the paper does not specify a rule): parameters chosen so
    that sketched Ritz values, which are complex even for real spectra, are
    enclosed with margin; pinned against dense exp of sketched projected
    matrices in the tests.

z^(-1/2)  -- Stieltjes form z^(-1/2) = (2/pi) int_0^inf (z + s^2)^{-1} ds with
    s = c tan(theta), theta in (0, pi/2), N midpoint nodes:
    zeta_l = -c^2 tan^2(theta_l),  w_l = -(c/N) sec^2(theta_l),
    c = (lambda_lo lambda_hi)^(1/4) from a spectral interval.

phi_1(-t z)  -- the same Hankel contour: with phi_1(s) = (e^s - 1)/s,
    (1/2 pi i) int e^s / (s (s - s0)) ds = phi_1(s0) for a contour enclosing
    0 and s0 (the residues at 0 and s0; the part -1/s of phi_1 integrates to
    zero, and e^s/s decays on the contour's tails like e^s itself), so the
    nodes are exp_rule's and each weight is divided by its node's s = -t zeta.
    The contour passes s = 0 at distance P, as it passes the spectrum's end.

cos(t sqrt(z))  -- Cauchy integral on an ellipse around the spectral interval:
    z(theta) = c + h (rho e^{i theta} + e^{-i theta}/rho)/2, c = (lo+hi)/2,
    h = (hi-lo)/2, trapezoidal rule in theta_k = 2 pi (k + 1/2)/N:
    zeta_k = z(theta_k), w_k = f(zeta_k) z'(theta_k) / (i N).  cos(t sqrt z)
    is entire (its series has integer powers of z only), so any ellipse
    around the interval works.  For a point z whose ellipse coordinate
    |w(z)| (z = c + h (w + 1/w)/2, |w| >= 1) is below rho the truncation error
    falls like (|w(z)|/rho)^N, while the rounding of the sum grows with max |f|
    on the ellipse, which grows with rho.  The points that matter are the
    eigenvalues of the cycle's projected matrices: sketched Ritz values, which
    can fall slightly outside [lo, hi] (the sketched projection is oblique).
    Reading (``cos_sqrt_rho``): rho_min = exp(37/N) is the smallest ellipse with
    rho^-N below FP64 rounding; the rule takes the largest of the candidates
    rho_min (2/rho_min)^(j/16), j = 16 .. 0, whose growth t max_k |Im sqrt
    zeta_k| over its nodes stays within max(ln 100, the growth at rho_min), so
    max |f| on the ellipse grows at most to ~100 or not beyond that of rho_min.
    Small t sqrt(hi) gets rho = 2, which serves Ritz values out to |w| ~ 1.7
    (0.15 h beyond the ends) at 1e-14; large t sqrt(hi) keeps rho_min (measured:
    rule error <= 6e-12 on [lo, hi] for t sqrt(hi) <= 100 at N = 256, the
    default).

Nodes of the exp rule come in complex-conjugate pairs (u, -u); for real
matrices ``conjugate_half`` keeps the Im zeta > 0 half, and the caller doubles
the real part.

Rule error (``rule_error``): the restarted iteration with a fixed rule r
converges to r(A) b, so the rule adds at most |r - f| over the spectral region
to the error.  It is sampled at 256 points: exp at t z = 0 and t z geometric in
[1e-4, 1e4] (absolute error; f <= 1), z^(-1/2) at z geometric in [lo, hi]
(relative error), phi_1(-t z) as exp (absolute error; 0 < f <= 1), cos(t sqrt z)
at sqrt(z) uniform in [sqrt(lo), sqrt(hi)] (absolute error; |f| <= 1).
"""
import numpy as np

EXP_MAIN = (128, 3.0, 6.0, 45.0)
RULE_SAMPLES = 256


def exp_rule(t: float, N: int = EXP_MAIN[0], P: float = EXP_MAIN[1], mu: float = EXP_MAIN[2],
             L: float = EXP_MAIN[3]):
    """(zeta, w) complex arrays of length N with sum_l w_l/(zeta_l - z) ~ exp(-t z)."""
    U = np.sqrt((P + L) / mu)
    h = 2.0 * U / N
    u = -U + (np.arange(N) + 0.5) * h
    s = P - mu * u ** 2 + 2j * mu * u
    ds = -2.0 * mu * u + 2j * mu
    zeta = -s / t
    w = -h * ds * np.exp(s) / (2j * np.pi * t)
    return zeta, w


def invsqrt_rule(N: int, lam_lo: float, lam_hi: float):
    """(zeta, w) real arrays with sum_l w_l/(zeta_l - z) ~ z^(-1/2) for z near [lam_lo, lam_hi]."""
    c = (lam_lo * lam_hi) ** 0.25
    th = (np.arange(N) + 0.5) * (np.pi / 2) / N
    zeta = -(c * np.tan(th)) ** 2
    w = -(c / N) / np.cos(th) ** 2
    return zeta.astype(complex), w.astype(complex)


def phi1_rule(t: float, N: int = EXP_MAIN[0], P: float = EXP_MAIN[1], mu: float = EXP_MAIN[2],
              L: float = EXP_MAIN[3]):
    """(zeta, w) with sum_l w_l/(zeta_l - z) ~ phi_1(-t z): exp_rule's nodes, weights over s = -t zeta."""
    zeta, w = exp_rule(t, N, P, mu, L)
    return zeta, w / (-t * zeta)


COS_SQRT_N = 256


COS_RHO_CAP = 2.0
COS_RHO_STEPS = 16
COS_GROWTH = np.log(100.0)


def _ellipse(c, h, rho, theta):
    e = np.exp(1j * theta)
    return c + h * (rho * e + 1.0 / (rho * e)) / 2.0, 1j * h * (rho * e - 1.0 / (rho * e)) / 2.0


def cos_sqrt_rho(t: float, N: int, lam_lo: float, lam_hi: float) -> float:
    """The ellipse parameter rho of the cos(t sqrt z) rule (the reading in the module header)."""
    c, h = 0.5 * (lam_lo + lam_hi), 0.5 * (lam_hi - lam_lo)
    theta = 2.0 * np.pi * (np.arange(N // 2) + 0.5) / N       # the nodes with Im zeta > 0
    rho_min = np.exp(37.0 / N)
    cap = max(COS_RHO_CAP, rho_min)

    def growth(rho):
        return t * np.max(np.abs(np.sqrt(_ellipse(c, h, rho, theta)[0]).imag))

    bound = max(COS_GROWTH, growth(rho_min))
    for j in range(COS_RHO_STEPS, 0, -1):
        rho = rho_min * (cap / rho_min) ** (j / COS_RHO_STEPS)
        if growth(rho) <= bound:
            return rho
    return rho_min


def cos_sqrt_rule(t: float, N: int, lam_lo: float, lam_hi: float):
    """(zeta, w) with sum_l w_l/(zeta_l - z) ~ cos(t sqrt(z)) for z near [lam_lo, lam_hi]."""
    rho = cos_sqrt_rho(t, N, lam_lo, lam_hi)
    c, h = 0.5 * (lam_lo + lam_hi), 0.5 * (lam_hi - lam_lo)
    e = np.exp(2j * np.pi * (np.arange(N) + 0.5) / N)
    zeta = c + h * (rho * e + 1.0 / (rho * e)) / 2.0
    dz = 1j * h * (rho * e - 1.0 / (rho * e)) / 2.0
    w = np.cos(t * np.sqrt(zeta)) * dz / (1j * N)
    return zeta, w


def conjugate_half(zeta, w):
    """Keep the Im(zeta) > 0 member of every conjugate pair (the rule must be conjugate-symmetric)."""
    keep = zeta.imag > 0
    return zeta[keep], w[keep]


def rational_scalar(zeta, w, z):
    """Evaluate r(z) = sum_l w_l/(zeta_l - z) on an array of scalars."""
    z = np.asarray(z, dtype=complex)
    return (w[None, :] / (zeta[None, :] - z.reshape(-1, 1))).sum(axis=1).reshape(z.shape)


def rule_error(fun: str, zeta, w, half: bool, t: float = 1.0, spec=None) -> float:
    """Largest error of r(z) = sum_l w_l/(zeta_l - z) against f on the sample set described above."""
    J = RULE_SAMPLES
    if fun in ("exp", "phi1"):
        tz = np.concatenate([[0.0], 1e-4 * 1e8 ** (np.arange(J - 1) / (J - 2))])
        z = tz / t
        f = np.exp(-tz) if fun == "exp" else np.where(tz > 0, -np.expm1(-tz) / np.where(tz > 0, tz, 1.0), 1.0)
    elif fun == "cos_sqrt":
        lo, hi = spec
        sq = np.sqrt(lo) + (np.sqrt(hi) - np.sqrt(lo)) * np.arange(J) / (J - 1)
        z, f = sq ** 2, np.cos(t * sq)
    else:
        lo, hi = spec
        z = lo * (hi / lo) ** (np.arange(J) / (J - 1))
        f = 1.0 / np.sqrt(z)
    r = rational_scalar(zeta, w, z)
    r = 2.0 * r.real if half else r.real
    return float(np.max(np.abs(r / f - 1.0)) if fun == "invsqrt" else np.max(np.abs(r - f)))
