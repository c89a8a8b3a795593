"""Seeded synthetic inputs for the SU(2) heat-bath workloads.

This module is the only code that both the oracle side and the HIP side of the
tests and the benchmark use.  It draws inputs only (lattice extents, couplings,
seeds, arbitrary link configurations, alpha grids) and holds none of the
method's arithmetic: no Philox, no staple, no heat-bath, no plaquette.

Link configurations are float32 arrays of shape [V, 4, 4] indexed (site lex,
direction mu, quaternion component) with lex = x0 + L0*(x1 + L1*(x2 + L2*x3));
direction 3 is time.  Random unit quaternions come from normalised 4-D Gaussians
(numpy's generator), which is Haar on SU(2) but is not the library's hot start.
"""
import numpy as np

# Lattice workloads, each a plain description of shape, coupling and start.
WORKLOADS = {
    "su2_4x4x4x4_b2.3_cold": dict(dims=(4, 4, 4, 4), beta=2.3, seed=1, start=0, sweeps=100),
    "su2_32x32x32x32_hot": dict(dims=(32, 32, 32, 32), betas=(2.2, 2.3, 2.4, 2.5), seed=1,
                                start=1, sweeps=1000),
    "su2_64x64x64x64_b2.4_hot": dict(dims=(64, 64, 64, 64), beta=2.4, seed=1, start=1,
                                     sweeps=200),
}

# Extents a batched replica may take (L^4 lattices) and its coupling range.
REPLICA_EXTENTS = (8, 12, 16, 20, 24)
REPLICA_BETA_RANGE = (1.8, 2.8)


def volume(dims):
    return int(np.prod(np.asarray(dims, dtype=np.int64)))


def random_links(dims, seed, dtype=np.float32):
    """Haar-random unit quaternions on every link (normalised Gaussians)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((volume(dims), 4, 4))
    g /= np.linalg.norm(g, axis=2, keepdims=True)
    return g.astype(dtype)


def near_identity_links(dims, seed, eps, dtype=np.float32):
    """Unit quaternions within ~eps of the identity: an ordered-phase-like
    state where the local coupling alpha is large."""
    rng = np.random.default_rng(seed)
    V = volume(dims)
    q = np.zeros((V, 4, 4))
    q[..., 0] = 1.0
    q[..., 1:] = eps * rng.standard_normal((V, 4, 3))
    q /= np.linalg.norm(q, axis=2, keepdims=True)
    return q.astype(dtype)


def replica_table(n, seed):
    """n replicas: extent L uniform on REPLICA_EXTENTS, beta uniform on
    REPLICA_BETA_RANGE, replica seed = seed + 1 + r.  Returns a list of dicts."""
    rng = np.random.default_rng(seed)
    Ls = rng.choice(np.asarray(REPLICA_EXTENTS), size=n)
    betas = rng.uniform(REPLICA_BETA_RANGE[0], REPLICA_BETA_RANGE[1], size=n)
    return [dict(dims=(int(L),) * 4, beta=float(b), seed=int(seed) + 1 + r, start=1)
            for r, (L, b) in enumerate(zip(Ls, betas))]


def alpha_grid(n=4096, alpha_max=40.0):
    """Uniform grid of n local couplings alpha in [0, alpha_max]."""
    return np.linspace(0.0, alpha_max, n)


def random_alphas(n, seed, alpha_max=40.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, alpha_max, size=n)


# The learned proposal's network 1 -> 64 -> 64 -> 33 has 6433 parameters in the
# order W1 (64x1), b1 (64), W2 (64x64), b2 (64), W3 (33x64), b3 (33).
MLP_SHAPES = ((64, 1), (64,), (64, 64), (64,), (33, 64), (33,))


def mlp_init(seed):
    """Initial parameters (float32, flat): weights uniform in
    [-1/sqrt(fan_in), 1/sqrt(fan_in)], biases zero."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in MLP_SHAPES:
        if len(shape) == 2:
            bound = 1.0 / np.sqrt(shape[1])
            parts.append(rng.uniform(-bound, bound, size=shape).ravel())
        else:
            parts.append(np.zeros(shape))
    return np.concatenate(parts).astype(np.float32)
