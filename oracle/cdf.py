"""CDF targets of the heat-bath variable x0 (test infrastructure; NumPy/SciPy, FP64).

For the local coupling alpha = beta |w| the component x0 of X = U V^dag has
density proportional to sqrt(1 - x^2) exp(alpha x) on [-1, 1] (the local
conditional of the Wilson action, Eqs. (2), (3), (6)).  Its CDF is

    F_alpha(x) = int_{-1}^{x} sqrt(1 - t^2) exp(alpha (t - 1)) dt / Z_alpha,

and the learned proposal is trained on the knots y_j = F_alpha^{-1}(j / 32),
j = 0..32 (y_0 = -1, y_32 = +1).  This is the definition written out with a
library quadrature (scipy.integrate.quad, in theta with x = cos(theta), which
removes the square-root endpoint behaviour) and a library root finder
(scipy.optimize.brentq); no blocking, tables or interpolation.
"""
import numpy as np
from scipy import integrate, optimize

NSEG = 32


def _density_theta(theta, alpha):
    # sqrt(1 - x^2) dx with x = cos(theta) -> sin(theta)^2 dtheta
    return np.sin(theta) ** 2 * np.exp(alpha * (np.cos(theta) - 1.0))


def mass_above(theta, alpha):
    """int_{x = cos(theta)}^{1} ... = mass of x0 in [cos(theta), 1]."""
    val, _ = integrate.quad(_density_theta, 0.0, theta, args=(alpha,), epsabs=0.0, epsrel=1e-13,
                            limit=200)
    return val


def normaliser(alpha):
    """Z_alpha = int_{-1}^{1} sqrt(1 - t^2) exp(alpha (t - 1)) dt."""
    return mass_above(np.pi, alpha)


def cdf(x, alpha):
    """F_alpha(x)."""
    x = float(np.clip(x, -1.0, 1.0))
    return 1.0 - mass_above(np.arccos(x), alpha) / normaliser(alpha)


def knots(alpha, nseg=NSEG):
    """y_j = F_alpha^{-1}(j / nseg), j = 0..nseg."""
    Z = normaliser(alpha)
    y = np.empty(nseg + 1)
    y[0], y[nseg] = -1.0, 1.0
    for j in range(1, nseg):
        target = (1.0 - j / nseg) * Z  # mass above the knot
        th = optimize.brentq(lambda t: mass_above(t, alpha) - target, 0.0, np.pi,
                             xtol=1e-15, rtol=4 * np.finfo(float).eps, maxiter=200)
        y[j] = np.cos(th)
    return y


def knot_table(alphas, nseg=NSEG):
    return np.array([knots(a, nseg) for a in np.asarray(alphas, dtype=np.float64)])


def log_widths(knot_rows):
    """log of the segment widths y_{j+1} - y_j (the quantity the MLP fits)."""
    k = np.asarray(knot_rows, dtype=np.float64)
    return np.log(np.diff(k, axis=-1))
