"""Autocorrelation-corrected error of a Monte Carlo time series: the Gamma
method of U. Wolff, "Monte Carlo errors with less errors", Comput. Phys.
Commun. 156 (2004) 143, with its automatic summation window (S = 1.5) and its
bias correction of the summed autocovariance.  Host-side analysis of the
plaquette histories the sweep produces (the paper keeps such averages on the
device and analyses them afterwards, Sec. 2.4)."""
import numpy as np


def autocovariance(x):
    """Gamma(t) = 1/(N-t) sum_i (x_i - mean)(x_{i+t} - mean), t = 0..N-1."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    d = x - x.mean()
    f = np.fft.rfft(d, n=2 * n)
    ac = np.fft.irfft(f * np.conj(f), n=2 * n)[:n]
    return ac / (n - np.arange(n))


def gamma_method(x, S=1.5):
    """Returns (mean, error of the mean, tau_int, error of tau_int, W).

    tau_int(W) = 1/2 + sum_{t=1}^{W} rho(t); the window W is the first one at
    which exp(-W/tau_hat) - tau_hat/sqrt(W N) turns negative, with
    tau_hat = S / ln((2 tau_int + 1)/(2 tau_int - 1)).  The summed
    autocovariance C(W) = Gamma(0) + 2 sum_{t<=W} Gamma(t) gets the factor
    (1 + (2W + 1)/N); error = sqrt(C/N), tau_int = C / (2 Gamma(0)),
    d tau_int = tau_int sqrt(2 (2W + 1) / N)."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    if n < 4:
        raise ValueError("need at least 4 samples")
    g = autocovariance(x)
    if g[0] <= 0.0:
        return float(x.mean()), 0.0, 0.5, 0.0, 0
    rho = g / g[0]
    tau_cum = 0.5 + np.cumsum(rho[1:])
    w_opt = n - 1
    for w in range(1, n):
        tau = tau_cum[w - 1]
        if tau <= 0.5:
            w_opt = w
            break
        tau_hat = S / np.log((2.0 * tau + 1.0) / (2.0 * tau - 1.0))
        if np.exp(-w / tau_hat) - tau_hat / np.sqrt(w * n) < 0.0:
            w_opt = w
            break
    c = g[0] + 2.0 * g[1:w_opt + 1].sum()
    c *= 1.0 + (2.0 * w_opt + 1.0) / n
    c = max(c, 0.0)
    tau_int = c / (2.0 * g[0])
    return (float(x.mean()), float(np.sqrt(c / n)), float(tau_int),
            float(tau_int * np.sqrt(2.0 * (2.0 * w_opt + 1.0) / n)), int(w_opt))
