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

Nodes of the exp rule come in complex-conjugate pairs (u, -u); for real
matrices ``conjugate_half`` keeps the Im zeta > 0 half, and the caller doubles
the real part.

Rule error (``rule_error``): the restarted iteration with a fixed rule r
converges to r(A) b, so the rule adds at most |r - f| over the spectral region
to the error.  It is sampled at 256 points: exp at t z = 0 and t z geometric in
[1e-4, 1e4] (absolute error; f <= 1), z^(-1/2) at z geometric in [lo, hi]
(relative error).
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
    if fun == "exp":
        tz = np.concatenate([[0.0], 1e-4 * 1e8 ** (np.arange(J - 1) / (J - 2))])
        z, f = tz / t, np.exp(-tz)
    else:
        lo, hi = spec
        z = lo * (hi / lo) ** (np.arange(J) / (J - 1))
        f = 1.0 / np.sqrt(z)
    r = rational_scalar(zeta, w, z)
    r = 2.0 * r.real if half else r.real
    return float(np.max(np.abs(r - f)) if fun == "exp" else np.max(np.abs(r / f - 1.0)))
