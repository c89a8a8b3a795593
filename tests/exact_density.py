"""Exact target distribution of the heat-bath variable x0 (test-side).

Given the staple sum w with k = |w| and alpha = beta k, the local conditional
of the updated link is proportional to exp(beta Re Tr(U W^dag)/2) times the
Haar measure (Eqs. (2), (3), (6)); writing U = X V with V = w/k, the component
x0 of X has density proportional to sqrt(1 - x0^2) exp(alpha x0) on [-1, 1].

This module tabulates that CDF by composite Simpson quadrature in
theta (x0 = cos theta), which removes the square-root endpoint singularity,
and gives the closed forms used as pins:
  Z(alpha)  = pi I1(alpha) / alpha  (int sqrt(1-t^2) e^{alpha t} dt)
  E[x0]     = I2(alpha) / I1(alpha)
  alpha = 0: F(x) = 1/2 + (x sqrt(1-x^2) + arcsin x) / pi
"""
import numpy as np
from scipy import special


def mean_x0(alpha):
    alpha = np.asarray(alpha, dtype=np.float64)
    return special.ive(2, alpha) / special.ive(1, alpha)


def haar_cdf(x):
    x = np.clip(np.asarray(x, dtype=np.float64), -1.0, 1.0)
    return 0.5 + (x * np.sqrt(1.0 - x * x) + np.arcsin(x)) / np.pi


class X0Cdf:
    """CDF of x0 at a fixed alpha, tabulated on n Simpson panels in theta."""

    def __init__(self, alpha, n=200000):
        self.alpha = float(alpha)
        th = np.linspace(0.0, np.pi, 2 * n + 1)
        # integrand in theta: sin^2(theta) exp(alpha (cos theta - 1)), from theta=pi (x0=-1)
        f = np.sin(th) ** 2 * np.exp(self.alpha * (np.cos(th) - 1.0))
        h = th[1] - th[0]
        # cumulative Simpson on panel boundaries (even indices), integrating from theta = pi down
        fr = f[::-1]
        panel = (fr[0:-2:2] + 4.0 * fr[1:-1:2] + fr[2::2]) * h / 3.0
        cum = np.concatenate([[0.0], np.cumsum(panel)])
        self.Z = cum[-1]
        self.theta = th[::-1][::2]  # pi ... 0, matching cum
        self.F = cum / cum[-1]
        self.x = np.cos(self.theta)  # -1 ... 1, increasing

    def __call__(self, x):
        return np.interp(np.asarray(x, dtype=np.float64), self.x, self.F)

    def inverse(self, u):
        return np.interp(np.asarray(u, dtype=np.float64), self.F, self.x)


def kp_accept_probability(alpha, n=400000):
    """Probability that one Kennedy-Pendleton attempt is accepted:
    E[sqrt(1 - s)] for s = G/(2 alpha), G ~ Gamma(3/2, 1), with s > 1 rejected."""
    from scipy import integrate, stats
    g = stats.gamma(1.5)
    val, _ = integrate.quad(lambda s: np.sqrt(1.0 - s) * g.pdf(2.0 * alpha * s) * 2.0 * alpha,
                            0.0, 1.0, limit=400)
    return val


def creutz_accept_probability(alpha):
    """Probability that one Creutz attempt is accepted: the target's mass
    pi I1(alpha) / alpha over the proposal's 2 sinh(alpha) / alpha."""
    alpha = np.asarray(alpha, dtype=np.float64)
    return np.pi * special.ive(1, alpha) / -np.expm1(-2.0 * alpha)


def kp_accept_closed_form(alpha):
    """The same for Kennedy-Pendleton in closed form: the accepted mass
    (pi / 2) I1(alpha) e^-alpha / alpha over the Gamma(3/2) proposal's
    Gamma(3/2) / (sqrt(2) alpha^(3/2)), i.e. sqrt(2 pi alpha) I1(alpha) e^-alpha."""
    alpha = np.asarray(alpha, dtype=np.float64)
    return np.sqrt(2.0 * np.pi * alpha) * special.ive(1, alpha)
