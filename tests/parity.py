"""Comparison helpers for HIP-vs-oracle parity.

A link update is an FP32 computation on the GPU and an FP64 one (with FP32
storage and an FP32 accept test) in the oracle, so updated links agree to
about 1e-6.  The one place where rounding can change a result by O(1) is the
Kennedy-Pendleton accept test: where u3^2 and 1 - lambda^2 differ by less than
the rounding of either side, the two may decide differently (a "flip").  A
mismatch is accepted as a flip only if the oracle reports a decision margin
below FLIP_MARGIN at that link; every other link must agree to LINK_TOL.
"""
import numpy as np

LINK_TOL = 1e-5      # per-component agreement of updated links
FLIP_MARGIN = 1e-5   # |u3^2 - (1 - lambda^2)| below which rounding may flip a decision
UNIT_TOL = 1e-6      # |q.q - 1| on every stored link


def compare_links(gpu, ora, margin=None):
    """gpu, ora: [..., 4] arrays; margin: oracle decision margins per link
    (same leading shape) or None.  Returns (n_flips, max_err_other)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ora = np.asarray(ora, dtype=np.float64)
    err = np.max(np.abs(gpu - ora), axis=-1)
    bad = err > LINK_TOL
    if margin is None:
        flips = np.zeros_like(bad)
    else:
        flips = bad & (np.asarray(margin) < FLIP_MARGIN)
    unexplained = bad & ~flips
    assert not np.any(unexplained), (
        f"{int(unexplained.sum())} links differ by more than {LINK_TOL} with a decision margin "
        f">= {FLIP_MARGIN}; worst {float(err[unexplained].max())}")
    other = err[~flips]
    return int(flips.sum()), float(other.max()) if other.size else 0.0


def unitarity_error(U):
    U = np.asarray(U, dtype=np.float64)
    return float(np.max(np.abs(np.sum(U * U, axis=-1) - 1.0)))


def parity_of(dims):
    V = int(np.prod(dims))
    x = np.array(np.unravel_index(np.arange(V), tuple(dims)[::-1]))
    return x.sum(axis=0) % 2


# ---------------------------------------------------------------------------
# How far FP32 rounding can move one updated link (Sec. 2.4, Eqs. (5)-(7)).
#
# The kernel forms the staple sum w in FP32 (each of the six staple terms a
# product of three unit quaternions, so |w| <= 6 and its rounding error is a
# few tens of eps = 2^-24 in absolute size), then V = w/|w| and alpha = beta|w|:
# both carry the error of w divided by k = |w|.  From lambda^2 it forms
# x0 = 1 - 2 lambda^2 and |a| = 2 sqrt(lambda^2 (1 - lambda^2)); a relative
# error r of lambda^2 moves x0 by 2 lambda^2 r and |a| by
# r sqrt(lambda^2 / (1 - lambda^2)) |1 - 2 lambda^2|, which grows without
# bound as x0 -> -1.  So an updated link can differ from the FP64 oracle's by
# about eps * cond with
#     cond = (1 + 6/k) (1 + kappa_x),  kappa_x = 2 lambda^2 + sqrt(lambda^2 / (1 - lambda^2)),
# lambda^2 = (1 - x0)/2.  A well-conditioned link (k of order 1..6, x0 away
# from -1) has cond <= COND_REF and is held to LINK_TOL; beyond COND_REF the
# bar grows with cond: LINK_TOL * cond / COND_REF = 1e-6 cond ~ 17 eps cond.
# Inputs that themselves carry an error delta (links an earlier pass of the
# same sweep wrote) move w by up to 18 * 2 delta (18 links in six staples;
# the factor 2 turns the per-component maximum into a 4-norm bound), which
# reaches the link as that change over k times (2 + kappa_x).
# ---------------------------------------------------------------------------
COND_REF = 10.0


def conditioning(knorm, x0):
    """cond of each update from the oracle's staple norm k and accepted x0
    (x0 NaN: no draw was accepted -- the link was kept -- cond from k only).
    Returns (cond, kappa_x)."""
    k = np.asarray(knorm, dtype=np.float64)
    x = np.asarray(x0, dtype=np.float64)
    lam2 = np.where(np.isnan(x), 0.0, (1.0 - x) / 2.0)
    one_m = np.maximum(1.0 - lam2, 1e-300)
    kx = 2.0 * lam2 + np.sqrt(lam2 / one_m)
    with np.errstate(divide="ignore"):
        cond = (1.0 + 6.0 / k) * (1.0 + kx)
    return cond, kx


# The overrelaxation move V U^dag V (no draw) carries the staple direction V
# twice: its bar takes kappa_x = 2 in place of the draw's.
KAPPA_OVERRELAX = 2.0


def link_tolerance(knorm, x0, delta_in=0.0, kappa_x=None):
    """Per-link bar: LINK_TOL up to COND_REF, growing with cond beyond it, plus
    the reach of an input error delta_in (per-component maximum).  kappa_x
    given: used in place of the draw's (x0 is then ignored)."""
    k = np.asarray(knorm, dtype=np.float64)
    if kappa_x is None:
        cond, kx = conditioning(knorm, x0)
    else:
        kx = np.full(k.shape, float(kappa_x))
        with np.errstate(divide="ignore"):
            cond = (1.0 + 6.0 / k) * (1.0 + kx)
    with np.errstate(divide="ignore", invalid="ignore"):
        inherited = np.where(np.asarray(delta_in) > 0, 36.0 * np.asarray(delta_in) * (2.0 + kx) / k, 0.0)
    return LINK_TOL * np.maximum(1.0, cond / COND_REF) + inherited


def compare_links_conditioned(gpu, ora, margin, knorm, x0, delta_in=0.0, kappa_x=None):
    """As compare_links, with the per-link bar of link_tolerance.  Returns a
    dict of statistics: updates, flips (mismatches at an oracle decision
    margin below FLIP_MARGIN), links over LINK_TOL, the largest error among
    the others, and for the links over LINK_TOL their errors, k, x0 and
    error / bar."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ora = np.asarray(ora, dtype=np.float64)
    err = np.max(np.abs(gpu - ora), axis=-1)
    tol = link_tolerance(knorm, x0, delta_in, kappa_x)
    flips = (err > LINK_TOL) & (np.asarray(margin) < FLIP_MARGIN)
    over = (err > LINK_TOL) & ~flips
    unexplained = over & (err > tol)
    idx = np.flatnonzero(over)
    st = dict(n=int(err.size), flips=int(flips.sum()), over=int(over.sum()),
              max_err_rest=float(err[~flips & ~over].max()) if np.any(~flips & ~over) else 0.0,
              max_ratio=float(np.max(err[~flips] / tol[~flips])) if np.any(~flips) else 0.0,
              over_err=err[idx], over_k=np.asarray(knorm)[idx],
              over_x0=np.asarray(x0)[idx] if x0 is not None else None,
              over_ratio=err[idx] / tol[idx], unexplained=int(unexplained.sum()))
    return st


def staple_inputs(dims, lex, mu):
    """The 18 links (site lex, direction) that the Eq. (6) staple of U_mu(x)
    reads, for an array of sites lex: returns (lex' [n, 18], dir [n, 18])."""
    L = np.asarray(dims, dtype=np.int64)
    lex = np.asarray(lex, dtype=np.int64)
    x = np.stack([lex % L[0], (lex // L[0]) % L[1], (lex // (L[0] * L[1])) % L[2],
                  lex // (L[0] * L[1] * L[2])], axis=1)

    def lx(c):
        return c[:, 0] + L[0] * (c[:, 1] + L[1] * (c[:, 2] + L[2] * c[:, 3]))

    def sh(c, d, s):
        c = c.copy()
        c[:, d] = (c[:, d] + s) % L[d]
        return c

    sites, dirs = [], []
    xpm = sh(x, mu, 1)
    for nu in range(4):
        if nu == mu:
            continue
        xpn, xmn = sh(x, nu, 1), sh(x, nu, -1)
        xpm_mn = sh(xpm, nu, -1)
        for c, d in ((x, nu), (xpn, mu), (xpm, nu), (xmn, nu), (xmn, mu), (xpm_mn, nu)):
            sites.append(lx(c))
            dirs.append(np.full(len(lex), d))
    return np.stack(sites, axis=1), np.stack(dirs, axis=1)


def pass_index(parity, mu):
    """Position of pass (parity, mu) in a sweep: odd parity first, mu = 0..3."""
    return (1 - int(parity)) * 4 + int(mu)
