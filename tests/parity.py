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
